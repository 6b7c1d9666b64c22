"""Comparison of GPU ERIs with the oracle.

The bar is |gpu - oracle| <= 1e-12 Ha per ERI, absolute.  The double build of
the oracle computes each quartet in the orientation it is given, so for
quartets whose HRR moves a high angular momentum across a long bond its own
rounding can approach 1e-12 Ha.  A quartet that misses the bar against the
double oracle is therefore recomputed with the oracle's __float128 build (the
referee, itself pinned against the double build), and must meet the same
absolute bar against that."""
import numpy as np

import oracle as O

ABS_TOL = 1e-12


def check_quartets(shells, quartets, got, ref, offs, sizes, threads=8):
    """got/ref: concatenated per-quartet values in the same (user) order.
    Returns (max error after refereeing, number of quartets refereed)."""
    err = np.abs(got - ref)
    bad_elem = err > ABS_TOL
    if not bad_elem.any():
        return float(err.max()) if len(err) else 0.0, 0
    qid = np.repeat(np.arange(len(sizes)), sizes)
    bad_q = np.unique(qid[bad_elem])
    quad, qoff, qsz = O.eri_quad(shells, quartets[bad_q], n_threads=threads)
    worst = 0.0
    for k, t in enumerate(bad_q):
        g = got[offs[t]:offs[t] + sizes[t]]
        r = quad[qoff[k]:qoff[k] + qsz[k]]
        e = np.abs(g - r)
        assert np.all(e <= ABS_TOL), \
            "quartet %d (L=%s): GPU differs from the __float128 referee by %.3e" % (
                t, [int(shells["L"][s]) for s in quartets[t]], e.max())
        worst = max(worst, float(e.max()))
    good = np.ones(len(err), dtype=bool)
    good[np.isin(qid, bad_q)] = False
    return max(worst, float(err[good].max()) if good.any() else 0.0), len(bad_q)
