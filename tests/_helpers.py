"""Shared helpers for the GPU parity tests (no test functions here)."""
import sys

import numpy as np

import oracle


def say(*a):
    """Name the case before a GPU step, flushed, so a failing run can be read."""
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def lib_to_oracle_perm():
    """perm[i_lib] = index of the same velocity vector in the oracle's order."""
    import paper_2604_17463_amd as P
    c, _ = P.velocity_set()
    oc, _, _ = oracle.lattice()
    lut = {tuple(v): i for i, v in enumerate(oc)}
    return np.array([lut[tuple(v)] for v in c])


def to_oracle(f_lib, perm):
    out = np.empty_like(f_lib)
    out[perm] = f_lib
    return out


def to_lib(f_orc, perm):
    return np.ascontiguousarray(f_orc[perm])


def rel_l2(a, b, ref=None):
    ref = b if ref is None else ref
    n = np.linalg.norm(ref)
    return np.linalg.norm(a - b) / (n if n > 0 else 1.0)


def deviation(f, rho0=1.0):
    _, w, _ = oracle.lattice()
    return f - (w * rho0)[:, None, None, None]
