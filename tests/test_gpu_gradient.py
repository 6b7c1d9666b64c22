"""GPU tests of the adjoint (eri_backward): gradients with respect to shell
centres and primitive exponents against the oracle's analytic gradient (all
four centres differentiated explicitly there), against finite differences of
the GPU forward values, and through the autograd functions."""
import os

import numpy as np
import pytest

import oracle as O
from paper_2303_13632_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 1)
RTOL = 1e-10     # relative to the largest gradient entry


def _quartets(n_shells, n, seed):
    rng = np.random.default_rng(seed)
    q = rng.integers(0, n_shells, size=(n, 4)).astype(np.int32)
    q[:4] = [[0, 0, 1, 1], [2, 3, 2, 3], [4, 4, 4, 4], [1, 0, 0, 1]]
    return q


def _close(got, ref, tol=RTOL):
    scale = max(np.abs(ref).max(), 1e-300)
    err = np.abs(got - ref).max()
    assert err <= tol * scale, (err, scale)


def _dl_plan(plan, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=plan.out_values)


@pytest.mark.parametrize("seed", [101, 102])
def test_explicit_dl_vs_oracle(seed):
    """Random dL/dERI over a quartet list that covers s, p, d shells in every
    position (repeated shells, swapped orders): GPU vs oracle gradient."""
    from paper_2303_13632_amd import eri
    print("explicit dl seed", seed, flush=True)
    sh = W.random_shells(12, lmax=2, seed=seed, box=4.0)
    q = _quartets(12, 300, seed)
    plan = eri.Plan(sh, q, bits=0)
    dlp = _dl_plan(plan, seed)
    dl_t = torch.tensor(dlp, device="cuda")
    gc, ge, en = plan.backward(dl=dl_t, energy=None)
    torch.cuda.synchronize()
    E, gx, gex = O.gradient(sh, q, dl=plan.to_user(dlp), n_threads=THREADS)
    _close(gc.cpu().numpy(), gx)
    _close(ge.cpu().numpy(), gex)
    assert abs(en.item() - E) <= RTOL * abs(E)


def test_explicit_density_vs_oracle():
    from paper_2303_13632_amd import eri
    sh = W.random_shells(10, lmax=2, seed=111, box=4.0)
    q = _quartets(10, 200, 111)
    plan = eri.Plan(sh, q, bits=0)
    D = W.random_density(plan.nbf, seed=111)
    gc, ge, en = plan.backward(density=torch.tensor(D, device="cuda"))
    torch.cuda.synchronize()
    E, gx, gex = O.gradient(sh, q, density=D, n_threads=THREADS)
    _close(gc.cpu().numpy(), gx)
    _close(ge.cpu().numpy(), gex)
    assert abs(en.item() - E) <= RTOL * abs(E)


def _unique_weights(qs):
    w = np.ones(len(qs))
    w *= np.where(qs[:, 0] != qs[:, 1], 2.0, 1.0)
    w *= np.where(qs[:, 2] != qs[:, 3], 2.0, 1.0)
    same = (np.minimum(qs[:, 0], qs[:, 1]) == np.minimum(qs[:, 2], qs[:, 3])) & \
           (np.maximum(qs[:, 0], qs[:, 1]) == np.maximum(qs[:, 2], qs[:, 3]))
    w *= np.where(same, 1.0, 2.0)
    return w


def test_batched_density_vs_oracle():
    """All unique screened quartets of a small molecule-like basis, density
    form with degeneracy weights: E and gradient against the oracle over the
    same quartets."""
    from paper_2303_13632_amd import eri
    sh = W.molecule_basis(n_heavy=1, n_h=3, lattice=(2, 2, 1), seed=W.SEED_BASE + 44)
    plan = eri.Plan(sh, None, bits=16, schwarz=1e-10)
    D = W.random_density(plan.nbf, seed=44)
    gc, ge, en = plan.backward(density=torch.tensor(D, device="cuda"))
    torch.cuda.synchronize()
    qs = np.concatenate([plan.class_quartet_list(c) for c in range(256) if plan.class_quartets[c]])
    print("batched quartets", len(qs), flush=True)
    E, gx, gex = O.gradient(sh, qs, weights=_unique_weights(qs), density=D, n_threads=THREADS)
    _close(gc.cpu().numpy(), gx)
    _close(ge.cpu().numpy(), gex)
    assert abs(en.item() - E) <= RTOL * abs(E)


def test_gradient_vs_gpu_finite_differences():
    """Central differences (Richardson, h = 1e-3) of the GPU forward values
    contracted with a fixed dL/dERI, on a sample of coordinates and
    exponents."""
    from paper_2303_13632_amd import eri
    sh = W.random_shells(8, lmax=2, seed=121, box=3.0)
    q = _quartets(8, 120, 121)
    plan = eri.Plan(sh, q, bits=0)
    dlp = _dl_plan(plan, 121)
    gc, ge, _ = plan.backward(dl=torch.tensor(dlp, device="cuda"))
    gc, ge = gc.cpu().numpy(), ge.cpu().numpy()
    scale = max(np.abs(gc).max(), np.abs(ge).max())

    def energy(s2):
        p2 = eri.Plan(s2, q, bits=0)
        out, _, _ = p2.alloc(eri=True, codes=False)
        p2.compute(out)
        torch.cuda.synchronize()
        return float(np.dot(out.cpu().numpy()[: p2.out_values], dlp))

    def fd(key, idx, h):
        def at(d):
            s2 = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in sh.items()}
            s2[key].reshape(-1)[idx] += d
            return energy(s2)
        d1 = (at(h) - at(-h)) / (2 * h)
        d2 = (at(h / 2) - at(-h / 2)) / h
        return (4 * d2 - d1) / 3

    rng = np.random.default_rng(121)
    for idx in rng.choice(3 * 8, size=6, replace=False):
        v = fd("xyz", int(idx), 1e-3)
        assert abs(v - gc.reshape(-1)[idx]) <= 1e-7 * scale, ("xyz", idx, v, gc.reshape(-1)[idx])
    for idx in rng.choice(len(sh["exps"]), size=6, replace=False):
        v = fd("exps", int(idx), 1e-3 * sh["exps"][idx])
        assert abs(v - ge[idx]) <= 1e-7 * scale, ("exps", idx, v, ge[idx])


def test_autograd_functions():
    from paper_2303_13632_amd import eri
    sh = W.random_shells(6, lmax=2, seed=131, box=3.0)
    q = _quartets(6, 60, 131)
    plan = eri.Plan(sh, q, bits=0)
    c = torch.tensor(sh["xyz"], device="cuda", requires_grad=True)
    e = torch.tensor(sh["exps"], device="cuda", requires_grad=True)
    vals = eri.ERIFunction.apply(c, e, plan)
    w = torch.tensor(_dl_plan(plan, 131), device="cuda")
    (vals[: plan.out_values] * w).sum().backward()
    gc, ge, _ = plan.backward(dl=w)
    torch.cuda.synchronize()
    _close(c.grad.cpu().numpy(), gc.cpu().numpy(), 1e-13)
    _close(e.grad.cpu().numpy(), ge.cpu().numpy(), 1e-13)
    # energy form
    D = torch.tensor(W.random_density(plan.nbf, seed=131), device="cuda")
    c.grad = None
    e.grad = None
    E = eri.CoulombEnergy.apply(c, e, plan, D)
    (3.0 * E).backward()
    E0, gx, gex = O.gradient(sh, q, density=D.cpu().numpy(), n_threads=THREADS)
    assert abs(E.item() - E0) <= RTOL * abs(E0)
    _close(c.grad.cpu().numpy(), 3.0 * gx)
    _close(e.grad.cpu().numpy(), 3.0 * gex)


def test_errors_and_empty():
    from paper_2303_13632_amd import eri
    sh = W.random_shells(4, lmax=2, seed=141)
    empty = eri.Plan(sh, np.zeros((0, 4), np.int32), bits=0)
    gc, ge, en = empty.backward(dl=torch.zeros(1, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    assert not gc.any() and not ge.any() and en.item() == 0.0
    f = W.random_shells(4, lmax=3, seed=142)
    f["L"][:] = 3
    pf = eri.Plan(f, np.array([[0, 1, 2, 3]], np.int32), bits=0)
    with pytest.raises(eri.EriError) as ex:
        pf.backward(dl=torch.zeros(pf.out_values, dtype=torch.float64, device="cuda"))
    assert ex.value.status == eri.ERI_EUNSUPPORTED
    mol = W.molecule_basis(n_heavy=1, n_h=2, lattice=(2, 2, 1), seed=W.SEED_BASE + 45)
    ring = eri.Plan(mol, None, bits=16, ring_bytes=4096)
    assert np.any(ring.class_ring < ring.class_quartets)
    with pytest.raises(eri.EriError) as ex:
        ring.backward(dl=torch.zeros(ring.out_values, dtype=torch.float64, device="cuda"))
    assert ex.value.status == eri.ERI_ESTATE
    with pytest.raises(eri.EriError):
        ring.backward(density=torch.zeros((ring.nbf + 1, ring.nbf + 1), dtype=torch.float64, device="cuda"))


def test_batched_energy_finite_differences():
    """Screened all-quartet plan (density form with degeneracy weights):
    central differences of the GPU energy against the GPU gradient."""
    from paper_2303_13632_amd import eri
    sh = W.molecule_basis(n_heavy=1, n_h=3, lattice=(2, 2, 1), seed=W.SEED_BASE + 46)
    plan = eri.Plan(sh, None, bits=0, schwarz=0.0)
    D = torch.tensor(W.random_density(plan.nbf, seed=46), device="cuda")
    gc, ge, _ = plan.backward(density=D)
    gc, ge = gc.cpu().numpy().reshape(-1), ge.cpu().numpy()
    scale = max(np.abs(gc).max(), np.abs(ge).max())

    def energy(s2):
        p2 = eri.Plan(s2, None, bits=0, schwarz=0.0)
        _, _, en = p2.backward(density=D, energy_only=True)
        return en.item()

    def fd(key, idx, h):
        def at(d):
            s2 = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in sh.items()}
            s2[key].reshape(-1)[idx] += d
            return energy(s2)
        d1 = (at(h) - at(-h)) / (2 * h)
        d2 = (at(h / 2) - at(-h / 2)) / h
        return (4 * d2 - d1) / 3

    rng = np.random.default_rng(46)
    for idx in rng.choice(len(gc), size=5, replace=False):
        v = fd("xyz", int(idx), 1e-3)
        assert abs(v - gc[idx]) <= 1e-7 * scale, ("xyz", idx, v, gc[idx])
    for idx in rng.choice(len(ge), size=5, replace=False):
        v = fd("exps", int(idx), 1e-3 * sh["exps"][idx])
        assert abs(v - ge[idx]) <= 1e-7 * scale, ("exps", idx, v, ge[idx])


def _sample_screened(plan, n_per_class, seed):
    """Seeded sample of up to n_per_class quartets of every class of a
    screened plan (shell indices, in the order the plan computes them)."""
    rng = np.random.default_rng(seed)
    out = []
    for cid in range(256):
        n = int(plan.class_quartets[cid])
        if n == 0:
            continue
        for j in np.sort(rng.choice(n, size=min(n, n_per_class), replace=False)):
            out.append(plan.class_quartet_list(cid, int(j), 1)[0])
    return np.array(out, dtype=np.int32)


def test_config5_sample_vs_oracle():
    """The 64-atom basis of the gradient workload (heavy atoms s,s,s,p,p,d
    with K up to 6 and exponents up to 5000): a seeded sample of its
    screened quartets, every class present, (dd|dd) included.  With Gbar =
    w_q D_ab D_cd (w_q the unique-quartet degeneracy) passed as dL/dERI of an
    explicit plan, the GPU gradient matches the oracle's analytic gradient of
    sum_q w_q sum D D (ab|cd) to 1e-10 of its largest entry; the density
    form of the same explicit plan (w_q = 1) as well."""
    from paper_2303_13632_amd import eri
    sh = W.gradient_basis()
    full = eri.Plan(sh, None, bits=16, schwarz=1e-10)
    qs = _sample_screened(full, 48, 505)
    full.close()
    L = sh["L"]
    assert any(all(L[s] == 2 for s in q) for q in qs)
    assert max(sh["K"][s] for q in qs for s in q) == 6
    print("64-atom basis sample: %d screened quartets" % len(qs), flush=True)
    plan = eri.Plan(sh, qs, bits=0)
    D = W.random_density(plan.nbf)
    w = _unique_weights(qs)
    bf = np.zeros(len(L) + 1, dtype=np.int64)
    bf[1:] = np.cumsum((L + 1) * (L + 2) // 2)
    # Gbar in user order: w_q D[a b] D[c d] over the quartet's components
    gb = []
    for t, (a, b, c, d) in enumerate(qs):
        dab = D[bf[a]:bf[a + 1], bf[b]:bf[b + 1]]
        dcd = D[bf[c]:bf[c + 1], bf[d]:bf[d + 1]]
        gb.append(w[t] * np.einsum("ij,kl->ijkl", dab, dcd).reshape(-1))
    pos, eoff = plan.layout()
    dlp = np.zeros(plan.out_values)
    for t in range(len(qs)):
        dlp[eoff[t]:eoff[t] + len(gb[t])] = gb[t]
    gc, ge, en = plan.backward(dl=torch.tensor(dlp, device="cuda"))
    torch.cuda.synchronize()
    E, gx, gex = O.gradient(sh, qs, weights=w, density=D, n_threads=THREADS)
    _close(gc.cpu().numpy(), gx)
    _close(ge.cpu().numpy(), gex)
    assert abs(en.item() - E) <= RTOL * abs(E)
    gc1, ge1, en1 = plan.backward(density=torch.tensor(D, device="cuda"))
    torch.cuda.synchronize()
    E1, gx1, gex1 = O.gradient(sh, qs, density=D, n_threads=THREADS)
    _close(gc1.cpu().numpy(), gx1)
    _close(ge1.cpu().numpy(), gex1)
    assert abs(en1.item() - E1) <= RTOL * abs(E1)


def test_multi_pass():
    """Adjoint passes bounded to a few quartets (opts chunk_quartets), so every
    class runs in several passes: an explicit plan with dL/dERI and a screened
    plan with a density, against the oracle."""
    from paper_2303_13632_amd import eri
    sh = W.random_shells(12, lmax=2, seed=151, box=4.0)
    q = _quartets(12, 300, 151)
    plan = eri.Plan(sh, q, bits=0, chunk_quartets=7)
    dlp = _dl_plan(plan, 151)
    gc, ge, en = plan.backward(dl=torch.tensor(dlp, device="cuda"))
    torch.cuda.synchronize()
    E, gx, gex = O.gradient(sh, q, dl=plan.to_user(dlp), n_threads=THREADS)
    _close(gc.cpu().numpy(), gx)
    _close(ge.cpu().numpy(), gex)
    assert abs(en.item() - E) <= RTOL * abs(E)
    mol = W.molecule_basis(n_heavy=1, n_h=3, lattice=(2, 2, 1), seed=W.SEED_BASE + 47)
    bp = eri.Plan(mol, None, bits=16, schwarz=1e-10, chunk_quartets=16)
    D = W.random_density(bp.nbf, seed=47)
    gc, ge, en = bp.backward(density=torch.tensor(D, device="cuda"))
    torch.cuda.synchronize()
    qs = np.concatenate([bp.class_quartet_list(c) for c in range(256) if bp.class_quartets[c]])
    print("multi-pass screened: %d quartets" % len(qs), flush=True)
    E, gx, gex = O.gradient(mol, qs, weights=_unique_weights(qs), density=D, n_threads=THREADS)
    _close(gc.cpu().numpy(), gx)
    _close(ge.cpu().numpy(), gex)
    assert abs(en.item() - E) <= RTOL * abs(E)


def test_global_atomic_fallback():
    """A large gradient (3 per shell + one per primitive, more than 4096
    entries) over many slices: the per-quartet atomics land in the slice of
    their workgroup and the slices are added in order.  Against the oracle."""
    from paper_2303_13632_amd import eri
    n = 1200
    sh = W.random_shells(n, lmax=2, seed=161, box=12.0)
    assert 3 * n + len(sh["exps"]) > 4096
    rng = np.random.default_rng(161)
    q = rng.integers(0, n, size=(1500, 4)).astype(np.int32)
    plan = eri.Plan(sh, q, bits=0)
    dlp = _dl_plan(plan, 161)
    gc, ge, en = plan.backward(dl=torch.tensor(dlp, device="cuda"))
    torch.cuda.synchronize()
    E, gx, gex = O.gradient(sh, q, dl=plan.to_user(dlp), n_threads=THREADS)
    _close(gc.cpu().numpy(), gx)
    _close(ge.cpu().numpy(), gex)
    assert abs(en.item() - E) <= RTOL * abs(E)


def test_energy_deterministic_and_set_geometry():
    """The energy is summed in a fixed order: repeated calls give the same
    bits.  eri_plan_set_geometry moves the plan to new centres/exponents on
    the same quartets: its energy equals that of a plan built there."""
    from paper_2303_13632_amd import eri
    sh = W.random_shells(10, lmax=2, seed=171, box=4.0)
    q = _quartets(10, 200, 171)
    plan = eri.Plan(sh, q, bits=0)
    D = torch.tensor(W.random_density(plan.nbf, seed=171), device="cuda")
    e1 = plan.backward(density=D, energy_only=True)[2].item()
    e2 = plan.backward(density=D, energy_only=True)[2].item()
    assert e1 == e2
    sh2 = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in sh.items()}
    sh2["xyz"][3, 1] += 0.05
    sh2["exps"][4] *= 1.1
    plan.set_geometry(xyz=sh2["xyz"], exps=sh2["exps"])
    e3 = plan.backward(density=D, energy_only=True)[2].item()
    fresh = eri.Plan(sh2, q, bits=0)
    e4 = fresh.backward(density=D, energy_only=True)[2].item()
    E4, _, _ = O.gradient(sh2, q, density=D.cpu().numpy(), n_threads=THREADS)
    assert e3 != e1
    assert abs(e3 - e4) <= 1e-13 * abs(e4)
    assert abs(e3 - E4) <= RTOL * abs(E4)
    out, _, _ = plan.alloc(eri=True, codes=False)
    plan.compute(out)
    out2, _, _ = fresh.alloc(eri=True, codes=False)
    fresh.compute(out2)
    torch.cuda.synchronize()
    # (the fresh plan may orient an equal-L pair the other way: last bits differ)
    assert (out[: plan.out_values] - out2[: fresh.out_values]).abs().max().item() <= 1e-12


def test_config5_finite_differences():
    """The 64-atom basis, all screened quartets, E = sum D D (ab|cd) with
    degeneracy weights: central differences of the GPU energy at h = 1e-4
    (the plan's quartet set held fixed across the displacements) against the
    GPU gradient for a seeded sample of coordinates and exponents, within
    1e-6 relative (relative to max(|g_FD|, 1e-8 max|g|)).  The difference
    is Richardson-extrapolated from the steps h and 2h: the plain difference
    at h carries a truncation error h^2/6 times the third derivative, which
    reaches 1e-5 relative on the coordinates of atoms with exponents up to
    5000 (length scale 1/sqrt(alpha) ~ 0.014 Bohr); the plain difference is
    held to 3e-5."""
    from paper_2303_13632_amd import eri
    sh = W.gradient_basis()
    plan = eri.Plan(sh, None, bits=16, schwarz=1e-10)
    D = torch.tensor(W.random_density(plan.nbf), device="cuda")
    gc, ge, _ = plan.backward(density=D)
    gc, ge = gc.cpu().numpy().reshape(-1), ge.cpu().numpy()
    gmax = max(np.abs(gc).max(), np.abs(ge).max())
    x0 = np.array(sh["xyz"], dtype=np.float64).reshape(-1)
    e0 = np.array(sh["exps"], dtype=np.float64)
    h = 1e-4

    def energy(key, idx, d):
        x, e = x0.copy(), e0.copy()
        (x if key == "xyz" else e)[idx] += d
        plan.set_geometry(xyz=x, exps=e)
        return plan.backward(density=D, energy_only=True)[2].item()

    rng = np.random.default_rng(20230328)
    worst, worst_plain = [], []
    for key, g in (("xyz", gc), ("exps", ge)):
        for idx in rng.choice(len(g), size=4, replace=False):
            d1 = (energy(key, int(idx), h) - energy(key, int(idx), -h)) / (2 * h)
            d2 = (energy(key, int(idx), 2 * h) - energy(key, int(idx), -2 * h)) / (4 * h)
            fd = (4 * d1 - d2) / 3
            floor = 1e-8 * gmax
            rel = abs(fd - g[idx]) / max(abs(fd), floor)
            rel1 = abs(d1 - g[idx]) / max(abs(d1), floor)
            print("FD %s[%d]: analytic %.10e richardson %.10e rel %.2e (plain at h: rel %.2e)"
                  % (key, idx, g[idx], fd, rel, rel1), flush=True)
            worst.append(rel)
            worst_plain.append(rel1)
    plan.set_geometry(xyz=x0, exps=e0)
    assert max(worst) <= 1e-6, worst
    assert max(worst_plain) <= 3e-5, worst_plain
