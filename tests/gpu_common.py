"""Helpers shared by the GPU parity tests (oracle caches, host <-> device copies)."""
import functools
import sys

import numpy as np
import pytest

import fio_inputs as fi
from oracle import bf as obf
from oracle import fio as ofio
from oracle import solve as osolve


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def fiohss():
    torch_cuda()
    import paper_2609_11520_amd as F
    F.lib()       # raises when the library is not built: no fallback path exists
    return F


def dev(a):
    """numpy (N,) / (N, k) complex -> column-major complex128 CUDA tensor (N, k)."""
    torch = torch_cuda()
    a = np.asarray(a, dtype=np.complex128)
    if a.ndim == 1:
        a = a[:, None]
    return torch.from_numpy(np.ascontiguousarray(a.T)).to("cuda").t()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def perr(a, b):
    """Parity error of a against the reference b, element by element: the larger of the largest
    per-column relative error ||a_c - b_c|| / ||b_c|| and max |a - b| / max |b| (vectors are one
    column).  No whole-block norm: one bad column or entry is not averaged away."""
    a = np.asarray(a)
    b = np.asarray(b)
    if a.ndim == 1:
        a, b = a[:, None], b[:, None]
    d = a - b
    nd, nb = np.linalg.norm(d, axis=0), np.linalg.norm(b, axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        col = np.where(nb > 0, nd / nb, np.where(nd > 0, np.inf, 0.0))
    mb = np.abs(b).max()
    ent = np.abs(d).max() / mb if mb > 0 else (np.inf if np.abs(d).max() > 0 else 0.0)
    return float(max(col.max(), ent))


def ecbf(a, b):
    """Section 5's relative error estimator of an approximation (e_cBF): ||a - b||_2 / ||b||_2 over
    the given (sampled) entries.  It measures the butterfly's interpolation error against the
    dense K, a quantity of the method, not GPU-vs-oracle parity (that is perr)."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def step(msg):
    print("[gpu-test]", msg, flush=True)
    sys.stdout.flush()


PHASES = {"sin16": ofio.PHASE_SIN16, "dft": ofio.PHASE_DFT, "sin8": ofio.PHASE_SIN8}


@functools.lru_cache(maxsize=8)
def oracle_bf(n, q, phase):
    return obf.BF1D(n, q, PHASES[phase])


def omega_np(seed):
    return lambda l, r, c: fi.omega(seed, l, r, c)


@functools.lru_cache(maxsize=8)
def oracle_hss(n, q, phase, tol, p, seed):
    from oracle import ulv as oulv
    B = oracle_bf(n, q, phase)
    h = osolve.build_hss_for_bf(B, omega_np(seed), tol, p=p)
    return h, oulv.factor(h)


def gpu_bf(F, n, q, phase, imported, precs=None):
    c0, c1 = PHASES[phase]
    precs = precs or (F.FIO_PREC_FP64,)
    if imported:
        return F.BF(n, q, c0, c1, precs=precs, factors=oracle_bf(n, q, phase).export_factors())
    return F.BF(n, q, c0, c1, precs=precs)


def hss_generators(h):
    """Oracle HSS generators in the hss_import layout (ranks, packed column-major blocks)."""
    ranks, parts = [], []
    for l in range(1, h.Lh + 1):
        ranks += list(h.rank[l])
    for l in range(1, h.Lh + 1):
        for j in range(2 ** l):
            parts.append(np.asarray(h.U[l][j]).ravel(order="F"))
    for l in range(0, h.Lh):
        for j in range(2 ** l):
            parts.append(np.asarray(h.B[l][j]).ravel(order="F"))
    for j in range(2 ** h.Lh):
        parts.append(np.asarray(h.D[j]).ravel(order="F"))
    return np.array(ranks, dtype=np.int32), np.concatenate(parts)
