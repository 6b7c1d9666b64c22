"""Host-side checks of the generated workgroup Rys kernels (no GPU): the
per-ERI table of 1D-factor offsets decodes to the Cartesian components of
each ERI (Sec. II-C, eq. 8: ERI = sum over nodes of Ix Iy Iz), every offset
stays inside its axis block of the LDS buffer, and the launch shape covers
every ERI with a buffer that fits the LDS."""
import importlib.util
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2303_13632_amd", "csrc")


def _codegen():
    spec = importlib.util.spec_from_file_location("eri_codegen_rys", os.path.join(CSRC, "codegen.py"))
    G = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(G)
    return G


@pytest.mark.parametrize("user", [(3, 3, 3, 3), (3, 2, 1, 0), (2, 2, 1, 1), (0, 3, 3, 2), (1, 1, 2, 1)])
def test_rys_factor_table(user):
    G = _codegen()
    cp = G.ClassPlan(*user)
    name = G.kernel_name("rys", cp.user)
    for real in ("double", "float"):
        _, src, fpq = G.emit_mode_RW(cp, name, real=real)
        body = re.search(r"%s_tab\[(\d+)\] = \{([^}]*)\}" % name, src, re.S)
        n = int(body.group(1))
        tab = [int(v) for v in body.group(2).replace("\n", " ").split(",") if v.strip()]
        assert n == cp.n_eriq == len(tab)
        a, b, c, d = cp.a, cp.b, cp.c, cp.d
        dims = (a + 1, b + 1, c + 1, d + 1)
        NI = dims[0] * dims[1] * dims[2] * dims[3]

        def decode(o):
            out = []
            for k in (3, 2, 1, 0):
                out.append(o % dims[k])
                o //= dims[k]
            return tuple(reversed(out))
        k = 0
        for ai in G.comps(a):
            for bi in G.comps(b):
                for ci in G.comps(c):
                    for di in G.comps(d):
                        v = tab[k]
                        ox, oy, oz = v & 1023, (v >> 10) & 1023, v >> 20
                        assert 0 <= ox < NI and NI <= oy < 2 * NI and 2 * NI <= oz < 3 * NI
                        for axis, o in enumerate((ox, oy - NI, oz - 2 * NI)):
                            assert decode(o) == (ai[axis], bi[axis], ci[axis], di[axis])
                        k += 1
        assert fpq > 3 * (cp.Ltot // 2 + 1) * n


@pytest.mark.parametrize("user", [(3, 3, 3, 3), (3, 3, 3, 2), (2, 2, 2, 2), (3, 1, 1, 0)])
def test_rys_launch_shapes(user):
    G = _codegen()
    cp = G.ClassPlan(*user)
    N = cp.Ltot // 2 + 1
    for suffix, budget, occ, nts, unroll, tag in G.RYSW_VARIANTS:
        for vb in (8, 4):
            NT, S, NB, NI = G.rysw_shape(cp, budget, vb, nts)
            assert NT % 64 == 0 and NT <= 1024 and NT * S >= cp.n_eriq
            assert NB >= 1 and (NB == 1 or NB * N * 3 * NI * vb <= budget)
            assert NB * 2 * N >= 1 and 3 * NI <= 1024
            # the LDS of one workgroup: the factor buffer (or the staged codes), the per
            # primitive quartet setup and the b_max reduction
            lds = max(NB * N * 3 * NI * vb, 4 * cp.n_eriq) + NB * (2 * N + 18) * 8 + NT // 64 * 8
            assert lds <= 160 * 1024
