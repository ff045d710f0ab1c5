"""Helpers shared by the GPU parity tests: run the HIP path and compare with the oracle."""

from __future__ import annotations

import sys

import numpy as np
import torch

import paper_2408_16847_amd as z3
from oracle import cpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def err_m(test, ref):
    """Per-m max-normalised error: max |test - ref| / max |ref| over (b1, b2, re/im)."""
    out = []
    for m in range(ref.shape[0]):
        r = np.concatenate([ref[m].real.ravel(), ref[m].imag.ravel()])
        t = np.concatenate([test[m].real.ravel(), test[m].imag.ravel()])
        den = np.abs(r).max()
        out.append(float(np.abs(t - r).max() / (den if den > 0 else 1.0)))
    return np.array(out)


def build(xyz, x, edges, w=None, cell_size=0.0):
    """GPU index over a host catalogue xyz [3, n] with values x [n] or [nmaps, n]."""
    xyz_d = torch.from_numpy(np.ascontiguousarray(xyz)).cuda()
    w_d = None if w is None else torch.from_numpy(np.ascontiguousarray(w, dtype=np.float64)).cuda()
    idx = z3.Index(xyz_d, edges, weights=w_d, cell_size=cell_size)
    idx.set_values(torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda())
    torch.cuda.synchronize()
    return idx


def perm(idx):
    return idx.perm().cpu().numpy()


def gpu_multipoles(idx, m_max, p0, p1, prec="fp64", norm="bin"):
    out = z3.accumulate(idx, m_max, p0, p1, prec=prec, norm=norm, want_w=True, want_counts=True,
                        want_idhash=True)
    A = out["A"].double().cpu().numpy()  # [m+1, 2, nb, P]
    a = A[:, 0] + 1j * A[:, 1]
    return (np.transpose(a, (2, 0, 1)), out["W"].cpu().numpy().T, out["counts"].cpu().numpy().T,
            out["idhash"].cpu().numpy().view(np.uint64).T)


def oracle_multipoles(xyz, x, w, edges, m_max, piv_idx):
    """Oracle raw multipoles for catalogue members piv_idx (original indices)."""
    return cpu.multipoles(xyz[:, piv_idx], xyz, w, x, edges, m_max, ids=True)


def normalise(a, W):
    Wb = W[:, None, :]
    return np.where(Wb > 0, a / np.where(Wb > 0, Wb, 1.0), 0.0)
