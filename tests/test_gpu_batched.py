"""GPU tests of plans over all unique Schwarz-screened quartets of a shell set
(one graph launch over class-sorted work): the screened set, every quartet
against the oracle, fused codes, the bounded output ring and graph replays."""
import os

import numpy as np
import pytest

import oracle as O
from paper_2303_13632_amd import workloads as W
from parity_util import check_quartets

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 1)
TAU = 1e-10


def small_molecule():
    # 8 sites on a jittered 3.5 Bohr lattice: 2 heavy (s,s,s,p,p,d; K 1-6;
    # exponents up to 5000) and 6 H (s,s,p) -- 30 shells, 465 pairs
    return W.molecule_basis(n_heavy=2, n_h=6, lattice=(2, 2, 2), seed=W.SEED_BASE + 33)


def _canon(q):
    a, b, c, d = (int(x) for x in q)
    p1, p2 = (max(a, b), min(a, b)), (max(c, d), min(c, d))
    return (p1, p2) if p1 >= p2 else (p2, p1)


def _all_quartets(plan):
    out = []
    for cid in range(256):
        n = int(plan.class_quartets[cid])
        if n:
            out.append((cid, plan.class_quartet_list(cid)))
    return out


@pytest.fixture(scope="module")
def molecule():
    from paper_2303_13632_amd import eri
    sh = small_molecule()
    plan = eri.Plan(sh, None, bits=16, schwarz=TAU)
    e, c, s = plan.alloc(eri=True, codes=True)
    plan.compute(e, c, s)
    torch.cuda.synchronize()
    return sh, plan, e.cpu().numpy(), c.cpu().numpy().astype(np.int32), s.cpu().numpy()


def test_screened_set(molecule):
    """The planned quartets are exactly the unique quartets with
    Q_ab Q_cd >= tau, Q from the oracle's diagonal integrals."""
    sh, plan, _, _, _ = molecule
    n = len(sh["L"])
    pairs = [(a, b) for a in range(n) for b in range(a + 1)]
    diag = np.array([[a, b, a, b] for a, b in pairs], dtype=np.int32)
    v, off, sizes = O.eri(sh, diag, n_threads=THREADS)
    Q = {}
    for k, (a, b) in enumerate(pairs):
        m = int(round(np.sqrt(sizes[k])))
        blk = v[off[k]:off[k] + sizes[k]].reshape(m, m)
        Q[(a, b)] = np.sqrt(np.max(np.abs(np.diag(blk))))
    keys = sorted(pairs)
    qv = np.array([Q[p] for p in keys])
    expected = set()
    near = set()
    for i, p1 in enumerate(keys):
        for j in range(i + 1):
            prod = qv[i] * qv[j]
            if prod >= TAU:
                expected.add((p1, keys[j]))
            if abs(prod - TAU) <= 1e-8 * TAU:
                near.add((p1, keys[j]))
    got = set()
    total = 0
    for cid, qs in _all_quartets(plan):
        for q in qs:
            got.add(_canon(q))
        total += len(qs)
    assert total == len(got), "a quartet is planned twice"
    assert (got ^ expected) <= near, (len(got - expected), len(expected - got))
    print("screened quartets: %d of %d unique" % (len(got), len(keys) * (len(keys) + 1) // 2))


def test_values_and_codes(molecule):
    sh, plan, vals, codes, scales = molecule
    assert np.all(plan.class_ring == plan.class_quartets)
    for cid, qs in _all_quartets(plan):
        n = len(qs)
        ref, roff, rsz = O.eri(sh, qs, n_threads=THREADS)
        lo, hi = plan.class_eri_off[cid], plan.class_eri_off[cid + 1]
        got = vals[lo:hi]
        check_quartets(sh, qs, got, ref, roff, rsz, THREADS)
        blk = np.concatenate([roff, [roff[-1] + rsz[-1]]]).astype(np.int64)
        oc, oe = O.compress(16, got, blk)
        q0 = plan.class_quartet_off[cid]
        assert np.array_equal(oe, scales[q0:q0 + n])
        assert np.array_equal(oc, codes[lo:hi])


def test_ring_keeps_last_window(molecule):
    """With a bound on the output, every quartet is still computed and
    written; the ring slot j mod R of each class holds the last quartet that
    maps there."""
    from paper_2303_13632_amd import eri
    sh, full, fvals, fcodes, fscales = molecule
    total = int(full.class_eri_off[256]) * 2
    plan = eri.Plan(sh, None, bits=16, schwarz=TAU, ring_bytes=total // 7, chunk_quartets=4096)
    assert np.any(plan.class_ring < plan.class_quartets)
    assert int(plan.class_eri_off[256]) * 2 <= total // 7 + 2 * 10000
    _, c, s = plan.alloc(eri=False, codes=True)
    plan.compute(None, c, s)
    torch.cuda.synchronize()
    codes = c.cpu().numpy().astype(np.int32)
    scales = s.cpu().numpy()
    for cid in range(256):
        n, r = int(plan.class_quartets[cid]), int(plan.class_ring[cid])
        if n == 0:
            continue
        m = int((full.class_eri_off[cid + 1] - full.class_eri_off[cid]) // n)
        for j in range(max(0, n - r), n):
            slot = j % r
            a = codes[plan.class_eri_off[cid] + slot * m: plan.class_eri_off[cid] + (slot + 1) * m]
            b = fcodes[full.class_eri_off[cid] + j * m: full.class_eri_off[cid] + (j + 1) * m]
            assert np.array_equal(a, b)
            assert scales[plan.class_quartet_off[cid] + slot] == fscales[full.class_quartet_off[cid] + j]


def test_graph_replays(molecule):
    """Replays of the captured graph, with eager work and synchronisations in
    between, reproduce the first result bit for bit."""
    from paper_2303_13632_amd import eri
    sh, full, fvals, fcodes, fscales = molecule
    plan = eri.Plan(sh, None, bits=16, schwarz=TAU, chunk_quartets=2048)
    _, c, s = plan.alloc(eri=False, codes=True)
    for k in range(4):
        c.zero_()
        s.zero_()
        x = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        _ = (x * 2).sum().item()
        plan.compute(None, c, s)
        torch.cuda.synchronize()
        assert np.array_equal(c.cpu().numpy().astype(np.int32), fcodes), k
        assert np.array_equal(s.cpu().numpy(), fscales), k


def test_molecule_full_size_sampled():
    """The 384-atom molecule-like basis (1536 shells, every unique quartet with
    Q_ab Q_cd >= 1e-10) at full size, with the benchmark's kernels and launch
    structure: tuned variants, one graph launch, int16 codes plus the FP64
    values, into rings of 24 GB of codes (96 GB of values).  Per class, 1024
    seeded ring slots of the last window are checked against the oracle's
    values of the quartets that own them: FP64 values within 1e-12 Ha, codes
    and scales bit-identical to the oracle's compressor fed those values, and
    decoded values within half a step of the oracle's."""
    from paper_2303_13632_amd import eri
    sh = W.molecule_basis(n_heavy=128, n_h=256)
    plan = eri.Plan(sh, None, bits=16, schwarz=TAU, ring_bytes=int(24e9))
    plan.tune(sample_quartets=65536, trials=2)
    print("molecule plan: %d quartets, %d ERIs" % (plan.n_quartets, plan.n_eri), flush=True)
    e, c, s = plan.alloc(eri=True, codes=True)
    plan.compute(e, c, s)
    torch.cuda.synchronize()
    cn = 1.0 / (2 ** 15 - 1)
    rng = np.random.default_rng(384)
    picks, code_idx, scale_idx, sizes = [], [], [], []
    for cid in range(256):
        n, r = int(plan.class_quartets[cid]), int(plan.class_ring[cid])
        if n == 0:
            continue
        m = int((plan.class_eri_off[cid + 1] - plan.class_eri_off[cid]) // r)
        for slot in np.sort(rng.choice(min(n, r), size=min(1024, n, r), replace=False)):
            j = int(slot) + r * ((n - 1 - int(slot)) // r)     # last quartet written to this slot
            picks.append(plan.class_quartet_list(cid, j, 1)[0])
            base = int(plan.class_eri_off[cid]) + int(slot) * m
            code_idx.append(np.arange(base, base + m))
            scale_idx.append(int(plan.class_quartet_off[cid]) + int(slot))
            sizes.append(m)
    picks = np.array(picks, dtype=np.int32)
    idx = torch.from_numpy(np.concatenate(code_idx)).cuda()
    vals = e[idx].cpu().numpy()
    codes = c[idx].cpu().numpy().astype(np.int32)
    scales = s[torch.from_numpy(np.array(scale_idx)).cuda()].cpu().numpy()
    del e, c, s, idx
    torch.cuda.empty_cache()
    ref, ref_off, ref_sizes = O.eri(sh, picks, n_threads=THREADS)
    assert np.array_equal(ref_sizes, sizes)
    print("molecule sample: %d quartets over %d classes" % (len(picks), int((plan.class_quartets > 0).sum())),
          flush=True)
    err, nref = check_quartets(sh, picks, vals, ref, ref_off, ref_sizes, THREADS)
    oc, oe = O.compress(16, vals, np.append(ref_off, len(vals)))
    assert np.array_equal(oe, scales)
    assert np.array_equal(oc, codes)
    # decoded values within half a step (plus the FP64 bar) of the oracle
    step = np.repeat(scales, sizes)
    bmax = np.repeat(scales / cn, sizes)
    assert np.all(np.abs(codes * step - vals) <= step / 2 + 4 * np.spacing(bmax))
    print("molecule sample: max |err| %.3e (%d quartets refereed in __float128)" % (err, nref))
