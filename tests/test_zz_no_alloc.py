"""eri_compute_noalloc (the entry point that allocates nothing) against
eri_compute, through the C ABI: screened plans (whose launch chunks are
staged in the library's static scratch array) and an explicit plan; two
calls in a row, the second on a smaller input; the size rule."""
import numpy as np
import pytest

from paper_2303_13632_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _both(plan, bits):
    e0, c0, s0 = plan.alloc(eri=True, codes=bits > 0)
    plan.compute(e0, c0, s0)
    e1, c1, s1 = plan.alloc(eri=True, codes=bits > 0)
    e1.fill_(np.nan)
    if c1 is not None:
        c1.fill_(7)
        s1.fill_(-1.0)
    plan.compute_noalloc(e1, c1, s1)
    torch.cuda.synchronize()
    n = plan.out_values
    assert torch.equal(e0[:n], e1[:n])
    if bits:
        assert torch.equal(c0[:n], c1[:n])
        assert torch.equal(s0[: plan.out_blocks], s1[: plan.out_blocks])
    return int(plan.n_quartets)


def test_noalloc_matches_compute():
    from paper_2303_13632_amd import eri
    big = W.molecule_basis(n_heavy=2, n_h=6, lattice=(2, 2, 2), seed=W.SEED_BASE + 33)
    p1 = eri.Plan(big, None, bits=16, schwarz=1e-10, chunk_quartets=1000)
    n1 = _both(p1, 16)
    small = W.molecule_basis(n_heavy=1, n_h=2, lattice=(2, 2, 1), seed=W.SEED_BASE + 34)
    p2 = eri.Plan(small, None, bits=16, schwarz=1e-10)
    n2 = _both(p2, 16)
    assert n2 < n1
    print("no-alloc: %d then %d quartets" % (n1, n2))
    parts = [W.class_case(cid, n_quartets=40) for cid in (0, 85, 170, 255)]
    shells, quartets = W.merge(parts)
    _both(eri.Plan(shells, quartets, bits=0), 0)


def test_noalloc_rejects_chunks_beyond_scratch():
    from paper_2303_13632_amd import eri
    sh = W.gradient_basis()
    p = eri.Plan(sh, None, bits=16, schwarz=1e-10, chunk_quartets=1 << 23)
    assert int(p.class_quartets.max()) > (1 << 22)
    _, c, s = p.alloc(eri=False, codes=True)
    with pytest.raises(eri.EriError) as ex:
        p.compute_noalloc(None, c, s)
    assert ex.value.status == eri.ERI_EUNSUPPORTED
