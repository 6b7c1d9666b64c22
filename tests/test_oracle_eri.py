"""Pins of the oracle's ERIs (eqs. 2-8) against facts it does not compute
itself: the (ss|ss) closed form, an independent numerical integration of
eq. 2, the 8-fold permutation symmetry of Sec. II-B, translation invariance,
the Schwarz inequality, parity zeros, and the __float128 instantiation."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import referee as RF
from paper_2303_13632_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def one_quartet(L, rng, K=(1,), box=6.0, erange=(0.1, 100.0)):
    Ls, Ks, xyz, ex, co = [], [], [], [], []
    for l in L:
        k = int(rng.choice(K))
        Ls.append(l); Ks.append(k)
        xyz.append(rng.uniform(0, box, 3))
        ex.append(np.exp(rng.uniform(np.log(erange[0]), np.log(erange[1]), k)))
        co.append(rng.uniform(0.1, 1.0, k))
    return W._pack(Ls, Ks, np.array(xyz), ex, co), np.array([[0, 1, 2, 3]], dtype=np.int32)


def test_ss_ss_closed_form():
    """(ss|ss) = 2 pi^(5/2)/(pq sqrt(p+q)) K_AB K_CD F_0(T), F_0 from erf."""
    sh, q = W.small_case(n_quartets=64)
    vals, _, _ = O.eri(sh, q)
    for t in range(64):
        idx = q[t]
        tot = 0.0
        A, B, C, D = (sh["xyz"][i] for i in idx)
        prims = [list(zip(sh["exps"][sh["off"][i]:sh["off"][i + 1]],
                          sh["coefs"][sh["off"][i]:sh["off"][i + 1]])) for i in idx]
        for a, ca in prims[0]:
            for b, cb in prims[1]:
                for c, cc in prims[2]:
                    for d, cd in prims[3]:
                        p, qq = a + b, c + d
                        P = (a * A + b * B) / p
                        Q = (c * C + d * D) / qq
                        rho = p * qq / (p + qq)
                        T = rho * np.sum((P - Q) ** 2)
                        F0 = 1.0 if T == 0 else 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))
                        kab = math.exp(-a * b / p * np.sum((A - B) ** 2))
                        kcd = math.exp(-c * d / qq * np.sum((C - D) ** 2))
                        nrm = (ca * RF.norm(a, 0) * cb * RF.norm(b, 0) * cc * RF.norm(c, 0)
                               * cd * RF.norm(d, 0))
                        tot += nrm * 2 * math.pi ** 2.5 / (p * qq * math.sqrt(p + qq)) * kab * kcd * F0
        assert vals[t] == pytest.approx(tot, rel=2e-14, abs=1e-16)


REFEREE_CLASSES = [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1),
                   (1, 1, 0, 0), (1, 0, 1, 0), (1, 1, 1, 0), (1, 1, 1, 1), (2, 0, 0, 0),
                   (0, 2, 1, 0), (2, 1, 0, 1), (2, 2, 0, 0), (1, 2, 2, 1), (2, 2, 2, 2),
                   (0, 0, 2, 2), (2, 0, 2, 0),
                   # f shells: every position, with s, p, d and f partners
                   (3, 0, 0, 0), (0, 3, 1, 0), (3, 1, 0, 0), (3, 0, 3, 0), (1, 3, 2, 0),
                   (3, 3, 0, 0), (0, 0, 3, 3), (3, 2, 1, 1), (2, 3, 3, 1), (3, 3, 3, 3)]


@pytest.mark.parametrize("L", REFEREE_CLASSES)
def test_against_numerical_integration(L):
    """Contracted quartets (K = 1 or 2) against direct numerical integration
    of eq. 2 (tests/referee.py)."""
    rng = np.random.default_rng(1000 + W.class_id(*L))
    for _ in range(2):
        sh, q = one_quartet(L, rng, K=(1, 2), box=4.0, erange=(0.15, 30.0))
        ref = RF.contracted_quartet(sh, q[0])
        got, _, _ = O.eri(sh, q)
        scale = max(np.max(np.abs(ref)), 1e-300)
        assert np.max(np.abs(got - ref)) <= 1e-12 * scale + 1e-15, (L, np.max(np.abs(got - ref)), scale)


def _perm_tensor(vals, L, perm):
    """Values of quartet (s0 s1 | s2 s3) reordered as the quartet perm."""
    n = [O.ncart(l) for l in L]
    t = vals.reshape(n)
    return t.transpose(perm).reshape(-1)


SYM = [((0, 1, 2, 3)), ((1, 0, 2, 3)), ((0, 1, 3, 2)), ((1, 0, 3, 2)),
       ((2, 3, 0, 1)), ((2, 3, 1, 0)), ((3, 2, 0, 1)), ((3, 2, 1, 0))]


def test_eightfold_symmetry_all_classes():
    """[ab|cd] = [ba|cd] = ... = [dc|ba] (Sec. II-B) for all 256 classes; each
    ordering walks a different path through eqs. 6-7."""
    rng = np.random.default_rng(7)
    for cid in range(256):
        L = W.class_of(cid)
        sh, q = one_quartet(L, rng, K=(1, 2), box=5.0, erange=(0.2, 20.0))
        base, _, _ = O.eri(sh, q)
        quarts = np.array([[q[0][p] for p in perm] for perm in SYM], dtype=np.int32)
        allv, off, sizes = O.eri(sh, quarts)
        scale = np.max(np.abs(base)) + 1e-300
        for k, perm in enumerate(SYM):
            v = allv[off[k]:off[k] + sizes[k]]
            # quartet perm has shells (s_perm0, ...); map back to (a,b,c,d) ordering
            inv = np.argsort(perm)
            back = _perm_tensor(v, [L[p] for p in perm], inv)
            assert np.max(np.abs(back - base)) <= 1e-12 * scale + 1e-15, (L, perm)


def test_translation_invariance():
    rng = np.random.default_rng(11)
    for cid in [0, 27, 85, 170, 255, 228, 99]:
        L = W.class_of(cid)
        sh, q = one_quartet(L, rng, K=(1, 2))
        a, _, _ = O.eri(sh, q)
        sh2 = dict(sh)
        sh2["xyz"] = sh["xyz"] + np.array([3.7, -12.25, 0.5])
        b, _, _ = O.eri(sh2, q)
        assert np.max(np.abs(a - b)) <= 1e-12 * (np.max(np.abs(a)) + 1e-300)


def test_schwarz_inequality():
    """(mn|ls)^2 <= (mn|mn)(ls|ls) for every component."""
    rng = np.random.default_rng(12)
    for cid in [5, 21, 42, 90, 150, 200, 255]:
        L = W.class_of(cid)
        sh, q = one_quartet(L, rng, K=(1, 2, 3))
        v, _, _ = O.eri(sh, q)
        dab, _, _ = O.eri(sh, np.array([[0, 1, 0, 1]], dtype=np.int32))
        dcd, _, _ = O.eri(sh, np.array([[2, 3, 2, 3]], dtype=np.int32))
        nab = O.ncart(L[0]) * O.ncart(L[1])
        ncd = O.ncart(L[2]) * O.ncart(L[3])
        dab = np.diag(dab.reshape(nab, nab))
        dcd = np.diag(dcd.reshape(ncd, ncd))
        bound = np.sqrt(np.outer(dab, dcd)).reshape(-1)
        assert np.all(np.abs(v) <= bound * (1 + 1e-12) + 1e-300)


def test_parity_zeros_one_centre():
    """All four shells on one centre: components whose total power on some
    axis is odd vanish by reflection symmetry (to rounding: the Gaussian
    product centre (aA + bA)/p rounds to within an ulp of A)."""
    rng = np.random.default_rng(13)
    for cid in [17, 65, 119, 255, 198]:
        L = W.class_of(cid)
        sh, q = one_quartet(L, rng, K=(1, 2))
        sh["xyz"][:] = sh["xyz"][0]
        v, _, _ = O.eri(sh, q)
        tol = 1e-13 * np.max(np.abs(v))
        comps = [O.components(l) for l in L]
        o = 0
        nz = 0
        for a in comps[0]:
            for b in comps[1]:
                for c in comps[2]:
                    for d in comps[3]:
                        odd = any((a[x] + b[x] + c[x] + d[x]) % 2 for x in range(3))
                        if odd:
                            assert abs(v[o]) <= tol
                        else:
                            nz += 1
                        o += 1
        assert nz > 0


def test_quad_referee_agrees():
    rng = np.random.default_rng(14)
    for cid in [0, 63, 127, 191, 255, 240, 15]:
        L = W.class_of(cid)
        sh, q = one_quartet(L, rng, K=(1, 2), box=10.0, erange=(0.1, 100.0))
        d, _, _ = O.eri(sh, q)
        qq, _, _ = O.eri_quad(sh, q)
        assert np.max(np.abs(d - qq)) <= 1e-13 * (np.max(np.abs(qq)) + 1e-300) + 1e-15


def test_paper_structural_facts():
    facts = json.load(open(os.path.join(GOLDEN, "paper_facts.json")))
    nc = O.ncart
    classes = [W.class_of(c) for c in range(256)]
    assert len(classes) == facts["n_generic_classes"]["value"]
    canon = [c for c in classes if c[0] >= c[1] and c[2] >= c[3] and nc(c[0]) * nc(c[1]) >= nc(c[2]) * nc(c[3])]
    assert len(canon) == facts["n_canonical_classes"]["value"]
    neriq = [nc(a) * nc(b) * nc(c) * nc(d) for a, b, c, d in classes]
    assert min(neriq) == facts["n_eriq_min"]["value"]
    assert max(neriq) == facts["n_eriq_max"]["value"]
    nrys = [(a + b + c + d) // 2 + 1 for a, b, c, d in classes]
    assert min(nrys) >= facts["n_rys_range"]["min"] and max(nrys) < facts["n_rys_range"]["max_exclusive"]
    for key, size in facts["i_buffer_size"]["values"].items():
        a, b, c, d = (int(x) for x in key.split(","))
        assert (a + 1) * (b + 1) * (c + 1) * (d + 1) * ((a + b + c + d) // 2 + 1) * 3 == size
