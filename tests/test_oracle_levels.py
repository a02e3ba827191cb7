"""Nested levels from the finest level's solves (Sec. 2.3): with one noise
vector per sample for all levels, a class's probe is the sum of its
sub-classes' probes, so each coarser level's estimate follows from the finest
solutions.  Pinned against the oracle's own direct estimate of every level
(its probes solved separately): equal up to the CG tolerance."""
import numpy as np
import pytest

import oracle
import workloads


@pytest.mark.parametrize("dims,p,ks,dilute,kind", [((4, 4, 4, 4), 1, (1, 2, 3), True, oracle.Z2_COMPLEX),
                                                   ((6, 4, 4, 4), 2, (1, 3), False, oracle.REAL_Z2)])
def test_levels_from_finest_solves_equal_direct(dims, p, ks, dilute, kind):
    U = workloads.random_links(dims, 0.4, 3, 3)
    cols, ncols = oracle.coloring_nested(dims, p, ks, oracle.NATURAL)
    lev = oracle.trace_levels(dims, 3, 0.3, U, p, cols, ncols, 5, 0, 2, kind, dilute, tol=1e-13)
    for l in range(len(ks)):
        d = oracle.trace(dims, 3, 0.3, U, p, cols[l], int(ncols[l]), 5, 0, 2, kind, dilute, tol=1e-13)
        assert abs(lev[l]["T"] - d["T"]) < 1e-10 * abs(d["T"]), (l, lev[l]["T"], d["T"])
        assert np.abs(lev[l]["per_sample"] - d["per_sample"]).max() < 1e-10 * abs(d["T"])
    # the finest level is the plain estimate, term by term
    d = oracle.trace(dims, 3, 0.3, U, p, cols[-1], int(ncols[-1]), 5, 0, 2, kind, dilute, tol=1e-13)
    assert np.abs(lev[-1]["tj"] - d["tj"]).max() < 1e-10 * np.abs(d["tj"]).max()


def test_levels_differ_from_each_other():
    """The identity is not vacuous: the levels' estimates differ (coarser
    classes leave more neighbours in one probe)."""
    dims, p = (4, 4, 4, 4), 1
    U = workloads.random_links(dims, 0.4, 3, 3)
    cols, ncols = oracle.coloring_nested(dims, p, (1, 3), oracle.NATURAL)
    lev = oracle.trace_levels(dims, 3, 0.3, U, p, cols, ncols, 5, 0, 1, oracle.Z2_COMPLEX, True)
    assert abs(lev[0]["T"] - lev[1]["T"]) > 1e-6 * abs(lev[1]["T"])
