"""Seeded synthetic inputs: shell lists and quartet lists.

This module holds no ERI arithmetic.  It only draws random shells and quartets;
the same arrays feed both the GPU library and the CPU oracle.

A shell set is a dict of numpy arrays:
    L     int32[n]      angular momentum (0..3 = s, p, d, f)
    K     int32[n]      number of primitives
    xyz   float64[n,3]  centre (Bohr)
    off   int64[n+1]    prefix offsets of each shell's primitives
    exps  float64[sum K] exponents
    coefs float64[sum K] contraction coefficients (multiply normalised primitives)
    atom  int32[n]      atom index of the shell (centre owner), for gradients
A quartet list is int32[nq, 4] of shell indices (a, b, c, d).

Workloads (distributions as stated for the paper's method; see the design notes
for the readings of unspecified details):
  * `random_class_quartets`: every quartet owns four independent shells with
    centres uniform in [0, 10)^3 Bohr, exponents log-uniform in [0.1, 100] and
    coefficients uniform in [0.1, 1]; K per shell either fixed or uniform over a
    set.  (ss|ss) with K = 3 and 4096 quartets is the small case; 65536 quartets
    per class with K in {1, 2, 3} over all 256 classes is the full case.
  * `molecule_basis`: a molecule-like basis of "heavy" atoms (s,s,s,p,p,d;
    K 1-6; exponents log-uniform [0.1, 5000]) and "H" atoms (s,s,p) on a jittered
    3.5 Bohr lattice.
  * `paper_lattice`: the paper's own benchmark system, 32 sites on a 4x4x2 cubic
    lattice of spacing 1 Angstrom, each with primitive s, p, d, f shells of
    exponent 1.5.
"""
import numpy as np

SEED_BASE = 20230323
ANGSTROM = 1.0 / 0.52917721092  # Bohr per Angstrom


def class_id(la, lb, lc, ld):
    return la * 64 + lb * 16 + lc * 4 + ld


def class_of(cid):
    return (cid >> 6) & 3, (cid >> 4) & 3, (cid >> 2) & 3, cid & 3


def ncart(L):
    return (L + 1) * (L + 2) // 2


def _log_uniform(rng, lo, hi, size):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=size))


def _pack(L, K, xyz, exps_list, coefs_list, atom=None):
    L = np.asarray(L, dtype=np.int32)
    K = np.asarray(K, dtype=np.int32)
    off = np.zeros(len(L) + 1, dtype=np.int64)
    off[1:] = np.cumsum(K)
    exps = np.concatenate(exps_list) if len(exps_list) else np.zeros(0)
    coefs = np.concatenate(coefs_list) if len(coefs_list) else np.zeros(0)
    if atom is None:
        atom = np.arange(len(L), dtype=np.int32)
    return {
        "L": L, "K": K, "xyz": np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3),
        "off": off, "exps": exps.astype(np.float64), "coefs": coefs.astype(np.float64),
        "atom": np.asarray(atom, dtype=np.int32),
    }


def random_class_quartets(la, lb, lc, ld, n_quartets, seed, k_choices=(1, 2, 3), k_fixed=None,
                          box=10.0, exp_range=(0.1, 100.0), coef_range=(0.1, 1.0)):
    """n_quartets quartets of one class, each with four fresh shells.

    Shell 4t+s is shell s (a, b, c, d) of quartet t; every shell is its own atom.
    """
    rng = np.random.default_rng(seed)
    n = 4 * n_quartets
    L = np.tile(np.array([la, lb, lc, ld], dtype=np.int32), n_quartets)
    if k_fixed is not None:
        K = np.full(n, int(k_fixed), dtype=np.int32)
    else:
        K = rng.choice(np.asarray(k_choices, dtype=np.int32), size=n)
    xyz = rng.uniform(0.0, box, size=(n, 3))
    tot = int(K.sum())
    exps = _log_uniform(rng, exp_range[0], exp_range[1], tot)
    coefs = rng.uniform(coef_range[0], coef_range[1], size=tot)
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = np.cumsum(K)
    shells = {
        "L": L, "K": K.astype(np.int32), "xyz": xyz, "off": off, "exps": exps, "coefs": coefs,
        "atom": np.arange(n, dtype=np.int32),
    }
    quartets = np.arange(n, dtype=np.int32).reshape(n_quartets, 4)
    return shells, quartets


def small_case(seed=SEED_BASE + 0, n_quartets=4096):
    """(ss|ss), K = 3 on every shell, 4096 quartets."""
    return random_class_quartets(0, 0, 0, 0, n_quartets, seed, k_fixed=3)


def class_case(cid, n_quartets=65536, seed=SEED_BASE + 1):
    """One class of the 256-class case (K uniform in {1,2,3})."""
    la, lb, lc, ld = class_of(cid)
    return random_class_quartets(la, lb, lc, ld, n_quartets, seed * 1000 + cid)


def merge(parts):
    """Concatenate several (shells, quartets) pairs into one shell set."""
    Ls, Ks, xyzs, exps, coefs, atoms, qs = [], [], [], [], [], [], []
    base = 0
    abase = 0
    for sh, q in parts:
        Ls.append(sh["L"]); Ks.append(sh["K"]); xyzs.append(sh["xyz"])
        exps.append(sh["exps"]); coefs.append(sh["coefs"])
        atoms.append(sh["atom"] + abase)
        qs.append(q + base)
        base += len(sh["L"])
        abase += int(sh["atom"].max()) + 1 if len(sh["atom"]) else 0
    L = np.concatenate(Ls)
    K = np.concatenate(Ks)
    off = np.zeros(len(L) + 1, dtype=np.int64)
    off[1:] = np.cumsum(K)
    shells = {"L": L, "K": K, "xyz": np.concatenate(xyzs), "off": off,
              "exps": np.concatenate(exps), "coefs": np.concatenate(coefs),
              "atom": np.concatenate(atoms).astype(np.int32)}
    return shells, np.concatenate(qs).astype(np.int32)


def molecule_basis(n_heavy=128, n_h=256, lattice=(8, 8, 6), spacing=3.5, jitter=0.3, seed=SEED_BASE + 3,
                   heavy_k=(1, 6), heavy_exp=(0.1, 5000.0), h_k=(1, 3), h_exp=(0.1, 100.0),
                   heavy_sites=None):
    """Molecule-like basis on a jittered cubic lattice.

    Heavy atoms carry shells s, s, s, p, p, d with K uniform in heavy_k and
    exponents log-uniform in heavy_exp; H atoms carry s, s, p with K uniform in
    h_k and exponents log-uniform in h_exp.  Coefficients uniform in [0.1, 1].
    Heavy sites are a seeded permutation of the lattice sites, or every site
    whose index is in `heavy_sites` when given.
    """
    rng = np.random.default_rng(seed)
    nx, ny, nz = lattice
    sites = np.array([(i, j, k) for i in range(nx) for j in range(ny) for k in range(nz)], dtype=np.float64)
    sites = sites[: n_heavy + n_h] * spacing
    sites = sites + rng.uniform(-jitter, jitter, size=sites.shape)
    n_sites = len(sites)
    if heavy_sites is None:
        perm = rng.permutation(n_sites)
        heavy = np.zeros(n_sites, dtype=bool)
        heavy[perm[:n_heavy]] = True
    else:
        heavy = np.zeros(n_sites, dtype=bool)
        heavy[np.asarray(heavy_sites)] = True
    L, K, xyz, ex, co, atom = [], [], [], [], [], []
    for a in range(n_sites):
        if heavy[a]:
            shells_l, krange, erange = (0, 0, 0, 1, 1, 2), heavy_k, heavy_exp
        else:
            shells_l, krange, erange = (0, 0, 1), h_k, h_exp
        for l in shells_l:
            k = int(rng.integers(krange[0], krange[1] + 1))
            L.append(l); K.append(k); xyz.append(sites[a]); atom.append(a)
            ex.append(_log_uniform(rng, erange[0], erange[1], k))
            co.append(rng.uniform(0.1, 1.0, size=k))
    return _pack(L, K, np.array(xyz), ex, co, atom)


def gradient_basis(seed=SEED_BASE + 4):
    """64-atom basis of the molecule-like type on a 4x4x4 jittered 3.5 Bohr
    lattice; sites whose index is divisible by 3 are heavy."""
    heavy = [i for i in range(64) if i % 3 == 0]
    return molecule_basis(n_heavy=len(heavy), n_h=64 - len(heavy), lattice=(4, 4, 4), seed=seed,
                          heavy_sites=heavy)


def random_shells(n, lmax=2, seed=SEED_BASE + 6, box=4.0, k_choices=(1, 2, 3), exp_range=(0.1, 100.0)):
    """n shells with L uniform in 0..lmax, K uniform in k_choices, centres
    uniform in [0, box)^3 Bohr, exponents log-uniform in exp_range,
    coefficients uniform in [0.1, 1]."""
    rng = np.random.default_rng(seed)
    L = rng.integers(0, lmax + 1, size=n)
    K = rng.choice(np.asarray(k_choices), size=n)
    xyz = rng.uniform(0.0, box, size=(n, 3))
    exps = [_log_uniform(rng, exp_range[0], exp_range[1], int(k)) for k in K]
    coefs = [rng.uniform(0.1, 1.0, size=int(k)) for k in K]
    return _pack(L, K, xyz, exps, coefs)


def random_density(nbf, seed=SEED_BASE + 5, sigma=0.1):
    """Random symmetric matrix with entries N(0, sigma)."""
    rng = np.random.default_rng(seed)
    D = rng.normal(0.0, sigma, size=(nbf, nbf))
    return np.ascontiguousarray(np.triu(D) + np.triu(D, 1).T)


def paper_lattice():
    """The paper's benchmark system: 4x4x2 sites at 1 Angstrom, each with
    primitive s, p, d and f shells of exponent 1.5 (coefficient 1)."""
    sites = np.array([(i, j, k) for i in range(4) for j in range(4) for k in range(2)],
                     dtype=np.float64) * ANGSTROM
    L, K, xyz, ex, co, atom = [], [], [], [], [], []
    for a, s in enumerate(sites):
        for l in range(4):
            L.append(l); K.append(1); xyz.append(s); atom.append(a)
            ex.append(np.array([1.5])); co.append(np.array([1.0]))
    return _pack(L, K, np.array(xyz), ex, co, atom)


def subset_shells(shells, quartets):
    """Return (shells', quartets') restricted to the shells the quartets use."""
    used = np.unique(quartets.reshape(-1))
    remap = -np.ones(len(shells["L"]), dtype=np.int64)
    remap[used] = np.arange(len(used))
    K = shells["K"][used]
    off = np.zeros(len(used) + 1, dtype=np.int64)
    off[1:] = np.cumsum(K)
    ex = np.concatenate([shells["exps"][shells["off"][s]:shells["off"][s + 1]] for s in used]) if len(used) else np.zeros(0)
    co = np.concatenate([shells["coefs"][shells["off"][s]:shells["off"][s + 1]] for s in used]) if len(used) else np.zeros(0)
    sh = {"L": shells["L"][used], "K": K, "xyz": shells["xyz"][used], "off": off, "exps": ex,
          "coefs": co, "atom": shells["atom"][used]}
    return sh, remap[quartets].astype(np.int32)
