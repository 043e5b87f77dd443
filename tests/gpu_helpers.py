"""Shared helpers for GPU parity tests (comparison with the FP64 oracle)."""
import math

import numpy as np

import oracle

WCA = 2.0 ** (1.0 / 6.0)


def banner(msg):
    print("[case] " + msg, flush=True)


def oracle_pp(eps=1.0, sigma=1.0, rc=2.5, shift=math.nan, caprad=0.0):
    return oracle.pair_params(eps, sigma, rc, shift, caprad)


def assert_forces_close(Fg, Fo, fscale, tol, what=""):
    """Normwise and per-particle condition-aware check:
    |dF_i| <= tol * sum_j |f_ij|   and   ||dF|| <= tol ||F||."""
    d = np.linalg.norm(Fg - Fo, axis=1)
    bound = tol * fscale + 1e-300
    bad = np.nonzero(d > bound)[0]
    assert bad.size == 0, "%s: %d particles beyond tol %g, worst ratio %g at %d" % (
        what, bad.size, tol, (d / bound).max(), int(np.argmax(d / bound)))
    nrm = np.linalg.norm(Fo)
    if nrm > 0:
        assert np.linalg.norm(Fg - Fo) / nrm <= tol, what


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def unwrap(state, box):
    return state["pos"] + state["image"] * np.asarray(box)[None, :]
