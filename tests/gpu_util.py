"""Shared helpers of the GPU parity tests (inputs to device, comparisons)."""
import sys

import numpy as np
import torch

DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_max(a, b) -> float:
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def rel_l2(a, b) -> float:
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def random_cart(n, g, seed, ghost_scale=1.0):
    """Random ghost values (unknowns zero) and random density."""
    rng = np.random.default_rng(seed)
    m = n + 1 + 2 * (g - 1)
    phi = rng.normal(size=(m, m, m)) * ghost_scale
    s = slice(g, g + n - 1)
    phi[s, s, s] = 0.0
    rho = rng.normal(size=(m, m, m))
    return phi, rho
