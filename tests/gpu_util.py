"""Helpers shared by the GPU tests: device transfers and floating-point bounds."""
import numpy as np

U64 = 2.0 ** -53


def dev(a):
    """numpy float64 array -> column-major float64 tensor on cuda:0."""
    import torch
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a[:, None]
    t = torch.from_numpy(np.ascontiguousarray(a.T)).to("cuda:0")
    return t.t()


def empty(rows, cols):
    import torch
    return torch.empty((cols, rows), dtype=torch.float64, device="cuda:0").t()


def host(t):
    return t.detach().cpu().numpy()


def sum_bound(abs_product, nterms, c=2.0):
    """Elementwise bound on the rounding error of a float64 sum of `nterms`
    products whose absolute values sum to `abs_product` (gamma_n * |A||B|)."""
    g = nterms * U64
    return c * g / (1 - g) * abs_product + 1e-300


def inst_dict(inst, max_rhs=None):
    return {"E": dev(inst.E), "W": dev(inst.W), "n_w": inst.n_w,
            "max_rhs": inst.R if max_rhs is None else max_rhs}
