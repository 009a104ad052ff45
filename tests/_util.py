"""Shared helpers of the tests (no method arithmetic here)."""
import numpy as np


def peak_rel_err(got, ref) -> float:
    """max_i |got - ref| / max_i |ref| (0 when both are all zero)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    peak = float(np.max(np.abs(ref))) if ref.size else 0.0
    err = float(np.max(np.abs(got - ref))) if ref.size else 0.0
    if peak == 0.0:
        return err
    return err / peak


def oracle_params(pp):
    """Oracle parameters with the same values as a binding Params object."""
    import oracle as O
    return O.OracleParams(depth=pp.depth if pp.depth > 0 else None, centers=tuple(pp.centers),
                          deltas=tuple(pp.deltas), weights=tuple(pp.weights), q=pp.q, r=pp.r,
                          eps=pp.eps, border=pp.border, lam=pp.lam, potts=pp.potts, block=pp.lm_block,
                          flat_tol=pp.flat_tol, gabor_lambda=pp.gabor_lambda,
                          gabor_sigma=pp.gabor_sigma, gabor_radius=pp.gabor_radius)
