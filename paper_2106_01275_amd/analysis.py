"""Figures of merit of the probed estimator from measured per-sample values
(arXiv:2106.01275, Sec. 4.2-4.3).  Plain host arithmetic on the per-sample
estimates T_s that trace_estimate / trace_multi return; nothing here touches
the GPU.

* variance v(.) of one sample estimate: the unbiased sample variance of T_s
  (complex values: the mean of |T_s - T|^2);
* speed-up over unprobed Hutchinson, eq. (11): v(B) / (m v(B o HH^T)), both
  variances per sample, m probing vectors (solves) per probed sample;
* speed-up over classical probing, eq. (12):
  v(B o H0 H0^T) m0 / (v(B o Hp Hp^T) mp);
* normalised relative error, eq. (13): sqrt(v(B o Hp Hp^T) mp / M) / |Tr(B)|,
  M the largest colour count among the colourings being compared.
With dilution every probing vector stands for n_dil solves; pass the number
of solves per sample as m to compare runs with different dilution.
"""
from __future__ import annotations

import numpy as np


def sample_variance(per_sample) -> float:
    """Unbiased variance of the per-sample estimates (complex allowed)."""
    t = np.asarray(per_sample)
    if t.size < 2:
        raise ValueError("need at least two samples")
    return float(np.sum(np.abs(t - t.mean()) ** 2) / (t.size - 1))


def speedup_over_hutchinson(var_plain: float, var_probed: float, m: int) -> float:
    """Eq. (11): v(P_p A^-1) / (m v((P_p A^-1) o H H^T))."""
    return var_plain / (m * var_probed)


def speedup_over_cp(var_cp: float, m0: int, var_p: float, mp: int) -> float:
    """Eq. (12): v(B o H0 H0^T) m0 / (v(B o Hp Hp^T) mp), H0 the (0, k)
    colouring's probes, Hp the (p, k) colouring's."""
    return (var_cp * m0) / (var_p * mp)


def normalized_relative_error(var: float, m_p: int, M: int, trace) -> float:
    """Eq. (13): sqrt(v m_p / M) / |Tr(P_n A^-1)|."""
    return float(np.sqrt(var * m_p / M) / abs(trace))
