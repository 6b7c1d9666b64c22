"""GPU checks of the FP32-mixed path (FP32 VRR/HRR; FP64 Boys, prefactors,
contraction and compression) against the oracle.

The target is 1e-7 Ha per ERI on every class.  FP32-mixed plans run FP32
recurrences for the classes listed in mixed_fp32_classes.json (measured
within 1e-8 Ha on another seeded sample of 4096 quartets per class) and the
FP64 kernels for the others; eri_plan_info.class_fp32 says which.  Asserted
here, on samples drawn with other seeds: every launch variant of every class
within 1e-7 Ha, the tuned full-size plan within 1e-7 Ha on 1024 sampled
quartets per class, and fused codes equal to the compressor applied to the
same (mixed-precision) doubles."""
import os

import numpy as np
import pytest

import oracle as O
from paper_2303_13632_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
N_PER_CLASS = 32
THREADS = min(16, os.cpu_count() or 1)
BAR = 1e-7


def _block_offsets(plan):
    off = []
    for cid in range(256):
        n = int(plan.class_quartets[cid])
        if n:
            m = int((plan.class_eri_off[cid + 1] - plan.class_eri_off[cid]) // n)
            off.append(plan.class_eri_off[cid] + m * np.arange(n))
    return np.concatenate(off + [[plan.n_eri]]).astype(np.int64)


def test_mixed_every_variant():
    """Every launch variant of every class (the autotuner may pick any), 32
    quartets per class: per class, the largest error over the variants is
    within 1e-7 Ha; each variant's fused codes equal the compressor applied
    to its own doubles."""
    from paper_2303_13632_amd import eri
    parts = [W.class_case(cid, n_quartets=N_PER_CLASS, seed=W.SEED_BASE + 71) for cid in range(256)]
    shells, quartets = W.merge(parts)
    ref, ref_off, sizes = O.eri(shells, quartets, n_threads=THREADS)
    plan = eri.Plan(shells, quartets, precision="mixed", bits=16)
    nv = plan.class_n_variants
    worst = np.zeros(256)
    for k in range(int(nv.max())):
        print("variant pass %d" % k, flush=True)
        v = np.where(nv > k, k, 0).astype(np.int32)
        plan.set_variants(v)
        e, c, s = plan.alloc(eri=True, codes=True)
        plan.compute(e, c, s)
        torch.cuda.synchronize()
        vals = e.cpu().numpy()[: plan.n_eri]
        got = plan.to_user(vals)
        assert np.all(np.isfinite(got)), k
        for cid in np.nonzero(v == k)[0]:
            lo = ref_off[cid * N_PER_CLASS]
            hi = ref_off[(cid + 1) * N_PER_CLASS - 1] + sizes[(cid + 1) * N_PER_CLASS - 1]
            worst[cid] = max(worst[cid], float(np.abs(got[lo:hi] - ref[lo:hi]).max()))
        # compression of the mixed values is exact (FP64 quantiser on the same doubles)
        off = _block_offsets(plan)
        oc, oe = O.compress(16, vals, off)
        assert np.array_equal(oc, c.cpu().numpy()[: plan.n_eri].astype(np.int32)), k
        assert np.array_equal(oe, s.cpu().numpy()[: plan.n_quartets]), k
    plan.set_variants(np.zeros(256, np.int32))
    fp32 = plan.class_fp32.astype(bool)
    order = np.argsort(-worst)
    print("FP32 classes: %d of 256; worst FP32 classes: %s" % (
        int(fp32.sum()), ", ".join("c%03d %.2e" % (c_, worst[c_]) for c_ in order if fp32[c_])[:400]))
    bad = [(int(c_), worst[c_]) for c_ in range(256) if worst[c_] > BAR]
    assert not bad, bad


def test_mixed_full_size_sampled():
    """The full 256-class workload (65536 quartets per class) as the benchmark
    runs it in FP32-mixed (tuned variants), FP64 values and int16 codes: 1024
    seeded quartets per class against the oracle, each class within 1e-7 Ha;
    their codes equal the compressor applied to their doubles."""
    from paper_2303_13632_amd import eri
    qpc = 65536
    parts = [W.class_case(cid, n_quartets=qpc) for cid in range(256)]
    shells, quartets = W.merge(parts)
    del parts
    plan = eri.Plan(shells, quartets, precision="mixed", bits=16)
    plan.tune(sample_quartets=qpc, trials=2)
    e, c, s = plan.alloc(eri=True, codes=True)
    plan.compute(e, c, s)
    torch.cuda.synchronize()
    print("mixed plan computed", flush=True)
    rng = np.random.default_rng(3030)
    npick = 1024
    pick = np.concatenate([cid * qpc + np.sort(rng.choice(qpc, size=npick, replace=False)) for cid in range(256)])
    ref, ref_off, sizes = O.eri(shells, quartets[pick], n_threads=THREADS)
    pos, eoff = plan.layout()
    idx = np.concatenate([np.arange(eoff[t], eoff[t] + n) for t, n in zip(pick, sizes)])
    ti = torch.from_numpy(idx).cuda()
    got = e[ti].cpu().numpy()
    codes = c[ti].cpu().numpy().astype(np.int32)
    scales = s[torch.from_numpy(pos[pick]).cuda()].cpu().numpy()
    del e, c, s, ti
    torch.cuda.empty_cache()
    err = np.abs(got - ref)
    qerr = np.maximum.reduceat(err, ref_off)
    worst = qerr.reshape(256, npick).max(axis=1)
    fp32 = plan.class_fp32.astype(bool)
    order = np.argsort(-worst)
    print("full-size FP32-mixed: %d FP32 classes; worst classes %s" % (
        int(fp32.sum()), ", ".join("c%03d %.2e" % (c_, worst[c_]) for c_ in order[:10])))
    blk = np.append(ref_off, len(got))
    oc, oe = O.compress(16, got, blk)
    assert np.array_equal(oe, scales)
    assert np.array_equal(oc, codes)
    bad = [(int(c_), worst[c_]) for c_ in range(256) if worst[c_] > BAR]
    assert not bad, bad
