"""GPU packed code stream (512-bit words of floor(512/n) n-bit codes, each
quartet on a new word): the packed bytes equal the oracle's packing of the
same fused codes, unpacking restores them, and the decompressed values are
code * eps within half a step of the FP64 values."""
import numpy as np
import pytest

import oracle as O
from paper_2303_13632_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("bits", [12, 10, 16, 20, 3, 7, 32])
def test_packed_stream(bits):
    from paper_2303_13632_amd import eri
    parts = [W.class_case(cid, n_quartets=9, seed=W.SEED_BASE + 81) for cid in (0, 21, 85, 170, 238, 255)]
    sh, q = W.merge(parts)
    plan = eri.Plan(sh, q, bits=bits)
    e, c, s = plan.alloc(eri=True, codes=True)
    plan.compute(e, c, s)
    off = []
    for cid in range(256):
        n = int(plan.class_quartets[cid])
        if n:
            m = int((plan.class_eri_off[cid + 1] - plan.class_eri_off[cid]) // n)
            off.append(plan.class_eri_off[cid] + m * np.arange(n))
    off = np.concatenate(off + [[plan.n_eri]]).astype(np.int64)
    woff = eri.packed_word_offsets(bits, off)
    d_off = torch.tensor(off, device="cuda")
    d_woff = torch.tensor(woff, device="cuda")
    packed = eri.pack(bits, c, d_off, d_woff)
    codes, vals = eri.unpack(bits, packed, d_off, d_woff, scales=s, codes=True, values=True)
    torch.cuda.synchronize()
    host_codes = c.cpu().numpy()[: plan.n_eri].astype(np.int64)
    ref, ref_woff = O.pack(bits, host_codes, off)
    assert np.array_equal(woff, ref_woff)
    got = packed.cpu().numpy().view(np.uint8)[: len(ref)]
    assert np.array_equal(got, ref)
    assert np.array_equal(codes.cpu().numpy()[: plan.n_eri], host_codes)
    x = e.cpu().numpy()[: plan.n_eri]
    eps = np.repeat(s.cpu().numpy()[: plan.n_quartets], np.diff(off))
    xt = vals.cpu().numpy()[: plan.n_eri]
    assert np.array_equal(xt, host_codes * eps)
    bmax = np.repeat(np.maximum.reduceat(np.abs(x), off[:-1]), np.diff(off))
    assert np.all(np.abs(x - xt) <= eps / 2 + 4 * np.spacing(bmax))


def _quartet_offsets(plan):
    off = []
    for cid in range(256):
        n = int(plan.class_quartets[cid])
        if n:
            m = int((plan.class_eri_off[cid + 1] - plan.class_eri_off[cid]) // n)
            off.append(plan.class_eri_off[cid] + m * np.arange(n))
    return np.concatenate(off + [[plan.n_eri]]).astype(np.int64)


FUSED_CLASSES = (0, 5, 21, 85, 95, 106, 170, 187, 231, 238, 245, 246, 250, 255)


@pytest.mark.parametrize("bits", [3, 7, 12, 16, 20, 32])
def test_fused_packed_stream(bits):
    """Plans with ERI_PLAN_PACKED write the packed stream from the ERI kernels
    (codes staged in LDS, no container array): its bytes equal the oracle's
    packing of the oracle's compression of the same doubles, every launch
    variant of every class at 12 and 20 bits (lane-per-quartet, slot and
    two-wavefront kernels, ragged workgroups; codes of several-chunk kernels
    over their own LDS at 12 bits, in dynamic LDS at 20)."""
    from paper_2303_13632_amd import eri
    parts = [W.class_case(cid, n_quartets=67, seed=W.SEED_BASE + 82) for cid in FUSED_CLASSES]
    sh, q = W.merge(parts)
    plan = eri.Plan(sh, q, bits=bits, packed=True)
    nv = plan.class_n_variants
    off = _quartet_offsets(plan)
    for k in range(int(nv.max()) if bits in (12, 20) else 1):
        print("bits %d variant pass %d" % (bits, k), flush=True)
        plan.set_variants(np.where(nv > k, k, 0).astype(np.int32))
        e, c, s = plan.alloc(eri=True, codes=True)
        plan.compute(e, c, s)
        torch.cuda.synchronize()
        vals = e.cpu().numpy()[: plan.n_eri]
        oc, oe = O.compress(bits, vals, off)
        ref, woff = O.pack(bits, oc, off)
        assert int(woff[-1]) == int(plan.class_word_off[256])
        got = c.cpu().numpy().view(np.uint8)[: len(ref)]
        assert np.array_equal(got, ref), (bits, k)
        assert np.array_equal(s.cpu().numpy()[: plan.n_quartets], oe), (bits, k)
