"""Shared helpers of the GPU tests: build the oracle's and the binding's
problem descriptions from one workload dict, move fields between host and
device, and compare results."""
import numpy as np
import torch

import oracle
import paper_1309_1720_amd as rd
import rd_inputs as ri


def problems(w: dict, nsteps: int | None = None, **over):
    """(oracle.Problem, rd.Problem) for workload dict ``w``."""
    w = dict(w, **over)
    if nsteps is not None:
        w["nsteps"] = nsteps
    params = ri.params_array(w["model"])
    return oracle.Problem.from_workload(w, params=params), rd.Problem.from_workload(w, params)


def dev(z, device="cuda"):
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device) for a in z]


def host(ts):
    torch.cuda.synchronize()
    return [t.detach().cpu().numpy() for t in ts]


def rel_linf(got, ref):
    """Max over fields of max|got - ref| / max|ref| (absolute if ref == 0)."""
    out = 0.0
    for g, r in zip(got, ref):
        scale = float(np.max(np.abs(r)))
        err = float(np.max(np.abs(np.asarray(g) - np.asarray(r))))
        out = max(out, err / scale if scale > 0 else err)
    return out


def gpu_step(p_rd, z, checkpoints=None):
    zt = dev(z)
    rd.step(p_rd, zt, checkpoints)
    return host(zt)


def crop_windows(nx, ny, reach, size=48):
    """Windows (x0, y0, w, h) at corners, edges and the centre of an nx x ny
    grid, and for each the slice of cells farther than ``reach`` from any
    window edge that is not a domain edge."""
    size = min(size, nx, ny)
    xs = sorted({0, max(0, nx // 2 - size // 2), nx - size})
    ys = sorted({0, max(0, ny // 2 - size // 2), ny - size})
    out = []
    for x0 in xs:
        for y0 in ys:
            lx = 0 if x0 == 0 else reach
            hx = size if x0 + size == nx else size - reach
            ly = 0 if y0 == 0 else reach
            hy = size if y0 + size == ny else size - reach
            out.append((x0, y0, size, size, (slice(ly, hy), slice(lx, hx))))
    return out


def oracle_on_crops(w, z0, nsteps, reach, size=48):
    """Oracle results on windows of a large grid (valid cells only)."""
    params = ri.params_array(w["model"])
    res = []
    for x0, y0, cw, ch, valid in crop_windows(w["nx"], w["ny"], reach, size):
        pc = oracle.Problem.from_workload(dict(w, nx=cw, ny=ch), params=params, x0=x0,
                                          nx_total=w["nx"])
        out = oracle.step(pc, [a[y0:y0 + ch, x0:x0 + cw] for a in z0], nsteps)
        res.append(((x0, y0, cw, ch, valid), out))
    return res
