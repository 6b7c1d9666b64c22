"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars: FP64 ERIs within 1e-12 Hartree absolute of the oracle (quartets that
miss it against the double oracle are refereed by its __float128 build, with
the same absolute bar); the fused codes and scales
bit-identical to the oracle's compressor fed the GPU's doubles; decompressed
values within half a quantisation step."""
import os

import numpy as np
import pytest

import oracle as O
from paper_2303_13632_amd import workloads as W
from parity_util import check_quartets

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_PER_CLASS = 67          # ragged against 64-lane and multi-slot workgroups
THREADS = min(16, os.cpu_count() or 1)


def _eri_gpu(shells, quartets, precision="fp64", bits=16):
    from paper_2303_13632_amd import eri
    plan = eri.Plan(shells, quartets, precision=precision, bits=bits)
    out_eri, out_codes, out_scales = plan.alloc(eri=True, codes=bits > 0)
    plan.compute(out_eri, out_codes, out_scales)
    torch.cuda.synchronize()
    vals = out_eri.cpu().numpy()[: plan.n_eri]
    codes = out_codes.cpu().numpy()[: plan.n_eri].astype(np.int32) if bits > 0 else None
    scales = out_scales.cpu().numpy()[: plan.n_quartets] if bits > 0 else None
    return plan, vals, codes, scales


def _blocks(sizes):
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    return off


@pytest.fixture(scope="module")
def all_classes():
    parts = [W.class_case(cid, n_quartets=N_PER_CLASS) for cid in range(256)]
    shells, quartets = W.merge(parts)
    print("oracle: %d quartets" % len(quartets), flush=True)
    ref, ref_off, sizes = O.eri(shells, quartets, n_threads=THREADS)
    return shells, quartets, ref, sizes


def test_all_classes_fp64_and_int16(all_classes):
    shells, quartets, ref, sizes = all_classes
    plan, vals, codes, scales = _eri_gpu(shells, quartets, bits=16)
    got = plan.to_user(vals)
    offs = _blocks(sizes)
    worst = []
    for c in range(256):
        qs = np.arange(c * N_PER_CLASS, (c + 1) * N_PER_CLASS)
        lo, hi = offs[qs[0]], offs[qs[-1] + 1]
        e, nref = check_quartets(shells, quartets[qs], got[lo:hi], ref[lo:hi], offs[qs] - lo, sizes[qs], THREADS)
        worst.append((e, c, nref))
    worst.sort(reverse=True)
    print("worst classes:", [(W.class_of(c), "%.2e" % e, n) for e, c, n in worst[:5]])
    # fused compression: codes and scales bit-identical to the oracle's compressor
    # applied to the GPU's own doubles, block = one quartet (plan order)
    blk = _blocks(np.repeat(np.diff(plan.class_eri_off) // np.maximum(plan.class_quartets, 1), plan.class_quartets))
    oc, oe = O.compress(16, vals, blk)
    assert np.array_equal(oe, scales)
    bad = np.nonzero(oc != codes)[0]
    if len(bad):
        qbad = np.searchsorted(blk, bad[0], side="right") - 1
        cbad = np.searchsorted(plan.class_quartet_off, qbad, side="right") - 1
        pytest.fail("%d codes differ; first in class %d %s" % (len(bad), cbad, W.class_of(int(cbad))))
    dec = O.decompress(codes, scales, blk)
    for b in range(len(blk) - 1):
        s = slice(blk[b], blk[b + 1])
        bmax = np.max(np.abs(vals[s]))
        if bmax < 1e-300:
            # eps = b_max c_n is subnormal or zero: it carries too few bits for
            # the eps/2 bound; the error is still at most b_max
            bound = bmax + 4 * np.spacing(bmax)
        else:
            # eps/2 plus the rounding of 1/eps and of q*eps
            bound = scales[b] / 2 + 4 * np.spacing(bmax)
        assert np.max(np.abs(dec[s] - vals[s])) <= bound


@pytest.mark.parametrize("bits", [8, 12, 32])
def test_fused_bit_widths(bits):
    parts = [W.class_case(cid, n_quartets=40) for cid in (0, 21, 85, 106, 170, 231, 255)]
    shells, quartets = W.merge(parts)
    plan, vals, codes, scales = _eri_gpu(shells, quartets, bits=bits)
    sizes = np.repeat(np.diff(plan.class_eri_off) // np.maximum(plan.class_quartets, 1), plan.class_quartets)
    blk = _blocks(sizes)
    oc, oe = O.compress(bits, vals, blk)
    assert np.array_equal(oe, scales)
    assert np.array_equal(oc, codes)


def test_small_case_ss_ss_k3():
    """(ss|ss), K = 3, 4096 quartets: every quartet against the oracle, with
    scale blocks of one quartet (fused) and of 64 quartets (standalone)."""
    shells, quartets = W.small_case()
    ref, _, sizes = O.eri(shells, quartets, n_threads=THREADS)
    plan, vals, codes, scales = _eri_gpu(shells, quartets, bits=16)
    got = plan.to_user(vals)
    check_quartets(shells, quartets, got, ref, _blocks(sizes), sizes, THREADS)
    # one value per quartet: each code is +-(2^15-1) or 0 at block = quartet
    assert np.all(np.isin(np.abs(codes), [0, 32767]))
    # scale blocks of 64 consecutive quartets (one wavefront's worth): the
    # standalone compressor over the GPU values, bit-exact against the
    # oracle's compressor, decoded values within half a step of the oracle
    from paper_2303_13632_amd import eri
    off = np.arange(0, len(got) + 64, 64, dtype=np.int64)
    off[-1] = len(got)
    dx = torch.from_numpy(got).cuda()
    c64, s64 = eri.compress(16, dx, torch.from_numpy(off).cuda())
    torch.cuda.synchronize()
    oc, oe = O.compress(16, got, off)
    assert np.array_equal(s64.cpu().numpy()[: len(off) - 1], oe)
    assert np.array_equal(c64.cpu().numpy().astype(np.int32), oc)
    step = np.repeat(oe, np.diff(off))
    assert np.all(np.abs(oc * step - ref) <= step / 2 + 4 * np.spacing(np.repeat(oe / (1.0 / 32767), np.diff(off)))
                  + 1e-12)
    assert len(np.unique(np.abs(oc))) > 100     # G = 64 resolves the values within a block


def test_degenerate_geometries():
    """All four centres equal (T = 0, parity zeros), very tight and very
    diffuse exponents, far-apart pairs (large T)."""
    rng = np.random.default_rng(99)
    parts = []
    for cid in (0, 5, 21, 64, 85, 150, 255, 27, 228):
        sh, q = W.class_case(cid, n_quartets=12, seed=777)
        sh["xyz"] = sh["xyz"].copy()
        sh["exps"] = sh["exps"].copy()
        n = len(sh["L"])
        sh["xyz"][0:16] = sh["xyz"][0]             # quartets 0..3: one centre
        sh["xyz"][16:24] = sh["xyz"][16] + np.array([0, 0, 40.0])  # far apart
        sh["exps"][: len(sh["exps"]) // 3] *= 50.0   # tight
        parts.append((sh, q))
    shells, quartets = W.merge(parts)
    ref, _, sizes = O.eri(shells, quartets, n_threads=THREADS)
    plan, vals, codes, scales = _eri_gpu(shells, quartets, bits=16)
    got = plan.to_user(vals)
    check_quartets(shells, quartets, got, ref, _blocks(sizes), sizes, THREADS)


def test_empty_plan():
    from paper_2303_13632_amd import eri
    sh, q = W.class_case(0, n_quartets=1)
    plan = eri.Plan(sh, q[:0], bits=16)
    assert plan.n_quartets == 0 and plan.n_eri == 0
    e, c, s = plan.alloc()
    plan.compute(e, c, s)
    torch.cuda.synchronize()


def test_standalone_compress_decompress():
    from paper_2303_13632_amd import eri
    rng = np.random.default_rng(5)
    sizes = rng.integers(1, 400, size=300)
    sizes[7] = 0
    off = _blocks(sizes)
    x = rng.standard_normal(off[-1]) * np.repeat(10.0 ** rng.uniform(-9, 2, size=300), sizes)
    x[off[3]:off[4]] = 0.0
    dx = torch.from_numpy(x).cuda()
    doff = torch.from_numpy(off).cuda()
    for bits in (4, 8, 12, 16, 24, 32):
        codes, scales = eri.compress(bits, dx, doff)
        out = eri.decompress(bits, codes, scales, doff)
        torch.cuda.synchronize()
        oc, oe = O.compress(bits, x, off)
        assert np.array_equal(scales.cpu().numpy()[: len(sizes)], oe)
        assert np.array_equal(codes.cpu().numpy().astype(np.int32), oc)
        assert np.array_equal(out.cpu().numpy(), O.decompress(oc, oe, off))


def test_full_size_sampled():
    """The full 256-class workload (65536 quartets per class) in the
    benchmark's launch configuration (autotuned variants): 96 seeded random
    quartets per class checked one by one against the oracle, codes of those
    quartets against the oracle's compressor."""
    from paper_2303_13632_amd import eri
    qpc = 65536
    parts = [W.class_case(cid, n_quartets=qpc) for cid in range(256)]
    shells, quartets = W.merge(parts)
    del parts
    plan = eri.Plan(shells, quartets, precision="fp64", bits=16)
    plan.tune(sample_quartets=qpc, trials=2)
    e, c, s = plan.alloc(eri=True, codes=True)
    plan.compute(e, c, s)
    torch.cuda.synchronize()
    rng = np.random.default_rng(2024)
    pick = np.concatenate([cid * qpc + np.sort(rng.choice(qpc, size=96, replace=False)) for cid in range(256)])
    ref, ref_off, sizes = O.eri(shells, quartets[pick], n_threads=THREADS)
    pos, eoff = plan.layout()
    idx = np.concatenate([np.arange(eoff[t], eoff[t] + n) for t, n in zip(pick, sizes)])
    got = e[torch.from_numpy(idx).cuda()].cpu().numpy()
    codes = c[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.int32)
    scales = s[torch.from_numpy(pos[pick]).cuda()].cpu().numpy()
    blk = _blocks(sizes)
    e, nref = check_quartets(shells, quartets[pick], got, ref, blk, sizes, THREADS)
    print("full-size sample: %d quartets, max |err| %.3e (%d refereed in __float128)" % (len(pick), e, nref))
    oc, oe = O.compress(16, got, blk)
    assert np.array_equal(oe, scales)
    assert np.array_equal(oc, codes)


def _scale_blocks(plan):
    """Value offsets of the plan's scale blocks (G consecutive quartets of a
    class in plan order; the last block of a class may be shorter)."""
    G = plan.scale_block
    off = []
    for cid in range(256):
        n = int(plan.class_quartets[cid])
        if n == 0:
            continue
        m = int((plan.class_eri_off[cid + 1] - plan.class_eri_off[cid]) // n)
        off.append(plan.class_eri_off[cid] + m * np.arange(0, n, G))
    return np.concatenate(off + [[plan.n_eri]]).astype(np.int64)


@pytest.mark.parametrize("case,G", [("ss_k3", 64), ("ss_k3", 1), ("fd_pp", 64), ("fd_pp", 7), ("fd_pp", 1)])
def test_scale_block(case, G):
    """Scale blocks of G quartets (eq. 9 over the block): codes and scales
    bit-identical to the oracle's compressor fed the GPU doubles over the same
    blocks; decoded values within half a step of the oracle's values; the
    codes do not depend on whether FP64 values are requested too."""
    from paper_2303_13632_amd import eri
    if case == "ss_k3":
        shells, quartets = W.small_case()
    else:
        shells, quartets = W.class_case(W.class_id(3, 2, 1, 1), n_quartets=200)
    ref, _, sizes = O.eri(shells, quartets, n_threads=THREADS)
    plan = eri.Plan(shells, quartets, precision="fp64", bits=16, scale_block=G)
    assert plan.scale_block == G and plan.out_blocks == -(-len(quartets) // G)
    e, c, s = plan.alloc(eri=True, codes=True)
    plan.compute(e, c, s)
    _, c2, s2 = plan.alloc(eri=False, codes=True)
    plan.compute(None, c2, s2)
    torch.cuda.synchronize()
    vals = e.cpu().numpy()[: plan.n_eri]
    codes = c.cpu().numpy()[: plan.n_eri].astype(np.int32)
    scales = s.cpu().numpy()[: plan.out_blocks]
    assert np.array_equal(codes, c2.cpu().numpy()[: plan.n_eri].astype(np.int32))
    assert np.array_equal(scales, s2.cpu().numpy()[: plan.out_blocks])
    got = plan.to_user(vals)
    check_quartets(shells, quartets, got, ref, _blocks(sizes), sizes, THREADS)
    blk = _scale_blocks(plan)
    oc, oe = O.compress(16, vals, blk)
    assert np.array_equal(oe, scales)
    assert np.array_equal(oc, codes)
    # decoded (plan order) against the oracle's values in plan order
    pos, eoff = plan.layout()
    ref_plan = np.empty(plan.n_eri)
    for t in range(len(quartets)):
        ref_plan[eoff[t]:eoff[t] + sizes[t]] = ref[_blocks(sizes)[t]:_blocks(sizes)[t] + sizes[t]]
    step = np.repeat(scales, np.diff(blk))
    bmax = step * 32767.0
    assert np.all(np.abs(codes * step - ref_plan) <= step / 2 + 4 * np.spacing(bmax) + 1e-12)
    if G == 64 and case == "ss_k3":
        assert len(np.unique(np.abs(codes))) > 100     # a block resolves the values within it


def _tiny_scale_case():
    """Lane-per-quartet, slot and two-wavefront classes whose quartets cycle
    through three magnitudes: normal; the a shell's coefficients times 1e-306
    (b_max around 1e-310, so 1/eps overflows at every width); times 1e-300
    (eps normal or subnormal depending on n).  Normal and tiny quartets share
    workgroups, so the fused kernels' divide path (eps subnormal) runs beside
    the multiply path."""
    parts = [W.class_case(cid, n_quartets=45, seed=W.SEED_BASE + 91)
             for cid in (W.class_id(1, 0, 1, 0), W.class_id(3, 2, 3, 2), W.class_id(3, 3, 3, 2), 255)]
    shells, quartets = W.merge(parts)
    coefs = shells["coefs"].copy()
    for t, (a, _, _, _) in enumerate(quartets):
        f = (1.0, 1e-306, 1e-300)[t % 3]
        coefs[shells["off"][a]:shells["off"][a + 1]] *= f
    shells["coefs"] = coefs
    return shells, quartets


@pytest.mark.parametrize("bits", [8, 16, 32])
def test_subnormal_scales(bits):
    """Fused codes and scales bit-identical to the oracle's compressor of the
    GPU doubles when some eps are subnormal (codes from x / eps), every launch
    variant at 16 bits; FP64 values within 1e-12 of the oracle."""
    from paper_2303_13632_amd import eri
    shells, quartets = _tiny_scale_case()
    plan = eri.Plan(shells, quartets, bits=bits)
    nv = plan.class_n_variants
    sizes = np.repeat(np.diff(plan.class_eri_off) // np.maximum(plan.class_quartets, 1), plan.class_quartets)
    blk = _blocks(sizes)
    ref, ref_off, rsizes = O.eri(shells, quartets, n_threads=THREADS)
    for k in range(int(nv.max()) if bits == 16 else 1):
        print("bits %d variant pass %d" % (bits, k), flush=True)
        plan.set_variants(np.where(nv > k, k, 0).astype(np.int32))
        e, c, s = plan.alloc(eri=True, codes=True)
        plan.compute(e, c, s)
        torch.cuda.synchronize()
        vals = e.cpu().numpy()[: plan.n_eri]
        codes = c.cpu().numpy()[: plan.n_eri].astype(np.int32)
        scales = s.cpu().numpy()[: plan.n_quartets]
        oc, oe = O.compress(bits, vals, blk)
        assert np.array_equal(oe, scales), (bits, k)
        assert np.array_equal(oc, codes), (bits, k)
        got = plan.to_user(vals)
        assert float(np.abs(got - ref).max()) <= 1e-12
    with np.errstate(divide="ignore", over="ignore"):
        inv = 1.0 / scales
    n_div = int(np.sum((scales > 0) & np.isinf(inv)))
    n_mul = int(np.sum(np.isfinite(inv) & (scales > 0)))
    print("bits %d: %d quartets through x/eps, %d through x*(1/eps)" % (bits, n_div, n_mul))
    assert n_div >= 40 and n_mul >= 40


def test_subnormal_scales_packed():
    """The packed stream (12-bit) of the same case: bytes equal to the
    oracle's packing of the oracle's compression of the GPU doubles."""
    from paper_2303_13632_amd import eri
    shells, quartets = _tiny_scale_case()
    plan = eri.Plan(shells, quartets, bits=12, packed=True)
    sizes = np.repeat(np.diff(plan.class_eri_off) // np.maximum(plan.class_quartets, 1), plan.class_quartets)
    blk = _blocks(sizes)
    e, c, s = plan.alloc(eri=True, codes=True)
    plan.compute(e, c, s)
    torch.cuda.synchronize()
    vals = e.cpu().numpy()[: plan.n_eri]
    oc, oe = O.compress(12, vals, blk)
    ref, _ = O.pack(12, oc, blk)
    assert np.array_equal(c.cpu().numpy().view(np.uint8)[: len(ref)], ref)
    assert np.array_equal(s.cpu().numpy()[: plan.n_quartets], oe)
