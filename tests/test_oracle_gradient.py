"""Pins of the oracle's analytic ERI gradient (the adjoint is not in the paper;
these checks rest on calculus and on exact identities of the Coulomb integral):

* central finite differences of the oracle's own ERIs, Richardson-extrapolated
  (error O(h^4)), for every centre coordinate and every exponent;
* translation invariance: the four centre derivatives of each integral sum to
  zero, and the oracle differentiates all four explicitly;
* Coulomb scaling: with normalised primitives, (ab|cd) at centres lambda R and
  exponents alpha / lambda^2 equals (ab|cd) / lambda, so
  sum_s R_s . dE/dR_s - 2 sum_k alpha_k dE/dalpha_k = -E exactly;
* the density form agrees with the explicit-Gbar form.
"""
import numpy as np
import pytest

import oracle as O
from paper_2303_13632_amd import workloads as W

THREADS = 8


def _case(seed, n_shells=6, n_q=10, lmax=2):
    sh = W.random_shells(n_shells, lmax=lmax, seed=seed, box=3.0)
    rng = np.random.default_rng(seed + 1)
    q = rng.integers(0, n_shells, size=(n_q, 4)).astype(np.int32)
    # repeated shells inside quartets exercise the same-centre paths
    q[0] = [0, 0, 1, 1]
    q[1] = [2, 3, 2, 3]
    q[2] = [4, 4, 4, 4]
    _, off, sizes = O.eri(sh, q, n_threads=THREADS)
    dl = rng.uniform(-1.0, 1.0, size=int(sizes.sum()))
    return sh, q, dl


def _energy(sh, q, dl):
    v, _, _ = O.eri(sh, q, n_threads=THREADS)
    return float(np.dot(v, dl))


def _fd(sh, q, dl, key, idx, h):
    def at(delta):
        s2 = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in sh.items()}
        s2[key].reshape(-1)[idx] += delta
        return _energy(s2, q, dl)
    d1 = (at(h) - at(-h)) / (2 * h)
    d2 = (at(h / 2) - at(-h / 2)) / h
    return (4 * d2 - d1) / 3


@pytest.mark.parametrize("seed", [11, 12])
def test_gradient_vs_finite_differences(seed):
    sh, q, dl = _case(seed)
    E, gx, ge = O.gradient(sh, q, dl=dl, n_threads=THREADS)
    assert abs(E - _energy(sh, q, dl)) <= 1e-13 * max(1.0, abs(E))
    scale = max(np.abs(gx).max(), np.abs(ge).max())
    used = np.unique(q)
    for s in used:
        for x in range(3):
            fd = _fd(sh, q, dl, "xyz", 3 * s + x, 1e-3)
            assert abs(fd - gx[s, x]) <= 1e-7 * scale, (s, x, fd, gx[s, x])
    for s in used:
        for k in range(sh["K"][s]):
            i = sh["off"][s] + k
            h = 1e-3 * sh["exps"][i]
            fd = _fd(sh, q, dl, "exps", i, h)
            assert abs(fd - ge[i]) <= 1e-7 * scale, (s, k, fd, ge[i])


@pytest.mark.parametrize("seed", [21, 22, 23])
def test_translation_invariance(seed):
    sh, q, dl = _case(seed, n_shells=8, n_q=24)
    _, gx, _ = O.gradient(sh, q, dl=dl, n_threads=THREADS)
    tot = gx.sum(axis=0)
    assert np.all(np.abs(tot) <= 1e-11 * np.abs(gx).max()), tot


@pytest.mark.parametrize("seed", [31, 32, 33])
def test_coulomb_scaling_identity(seed):
    sh, q, dl = _case(seed, n_shells=8, n_q=24)
    E, gx, ge = O.gradient(sh, q, dl=dl, n_threads=THREADS)
    virial = float(np.sum(sh["xyz"] * gx)) - 2.0 * float(np.dot(sh["exps"], ge))
    scale = float(np.abs(sh["xyz"] * gx).sum() + 2.0 * np.abs(sh["exps"] * ge).sum())
    assert abs(virial + E) <= 1e-12 * scale, (virial, -E)


def test_density_form_matches_dl_form():
    sh, q, _ = _case(41, n_shells=6, n_q=12)
    nbf = int(sum(O.ncart(int(l)) for l in sh["L"]))
    D = W.random_density(nbf, seed=41)
    bf = np.concatenate([[0], np.cumsum([O.ncart(int(l)) for l in sh["L"]])])
    blocks = []
    for a, b, c, d in q:
        Dab = D[bf[a]:bf[a + 1], bf[b]:bf[b + 1]]
        Dcd = D[bf[c]:bf[c + 1], bf[d]:bf[d + 1]]
        blocks.append(np.einsum("ij,kl->ijkl", Dab, Dcd).reshape(-1))
    dl = np.concatenate(blocks)
    w = np.linspace(0.5, 2.0, len(q))
    E1, g1, e1 = O.gradient(sh, q, weights=w, dl=dl, n_threads=THREADS)
    E2, g2, e2 = O.gradient(sh, q, weights=w, density=D, n_threads=THREADS)
    assert abs(E1 - E2) <= 1e-14 * max(1.0, abs(E1))
    assert np.allclose(g1, g2, rtol=0, atol=1e-14 * np.abs(g1).max())
    assert np.allclose(e1, e2, rtol=0, atol=1e-14 * np.abs(e1).max())


def test_empty():
    sh = W.random_shells(3, seed=5)
    E, gx, ge = O.gradient(sh, np.zeros((0, 4), np.int32), dl=np.zeros(0), n_threads=THREADS)
    assert E == 0.0 and not gx.any() and not ge.any()
