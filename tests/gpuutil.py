"""Helpers shared by the GPU tests: run workloads through the C interface and through the oracle."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev():
    import torch
    return torch.device("cuda:0")


def to_dev(x, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), device=dev(), dtype=dtype)


def gpu_plan(mesh, **opts):
    from paper_1804_01130_amd import Mesh, Plan, default_options
    gm = Mesh.from_arrays(mesh)
    return gm, Plan(gm, default_options(**opts))


def gpu_traced_step(plan, gm, alpha, phi, U, dt):
    import torch
    n, nf = gm.n_cells, gm.n_faces
    tr = {"vert_alpha": torch.full((8 * n,), float("nan"), device=dev(), dtype=torch.float64),
          "kind": torch.full((n,), -1, device=dev(), dtype=torch.int32),
          "iso": torch.full((n,), float("nan"), device=dev(), dtype=torch.float64),
          "rec": torch.full((7 * n,), float("nan"), device=dev(), dtype=torch.float64),
          "dV": torch.full((nf,), float("nan"), device=dev(), dtype=torch.float64),
          "alpha_raw": torch.full((n,), float("nan"), device=dev(), dtype=torch.float64),
          "iters": torch.zeros((n,), device=dev(), dtype=torch.int32)}
    out, st = plan.step(to_dev(alpha), to_dev(phi), to_dev(U), dt, stats=True, trace=tr)
    torch.cuda.synchronize()
    host = {k: v.cpu().numpy() for k, v in tr.items()}
    host["vert_alpha"] = host["vert_alpha"].reshape(-1, 8)
    host["rec"] = host["rec"].reshape(-1, 7)
    return out.cpu().numpy(), st, host


def gpu_trajectory(plan, w, steps, alpha0=None):
    import torch
    a = to_dev(w.alpha0 if alpha0 is None else alpha0)
    b = torch.empty_like(a)
    cache = {}
    for n in range(steps):
        key = 0 if w.steady else n
        if key not in cache:
            phi, U = w.phi_U(n)
            cache = {key: (to_dev(phi), to_dev(U))}
        tphi, tU = cache[key]
        plan.step(a, tphi, tU, w.dt, out=b)
        a, b = b, a
    torch.cuda.synchronize()
    return a.cpu().numpy()


def oracle_trajectory(om, w, steps, alpha0=None, opts=None):
    a = np.array(w.alpha0 if alpha0 is None else alpha0, copy=True)
    if w.steady:
        phi, U = w.phi_U(0)
        return om.run(a, phi, U, w.dt, steps, opts)
    for n in range(steps):
        phi, U = w.phi_U(n)
        a, _ = om.step(a, phi, U, w.dt, opts)
    return a
