"""Generator of the class-specialised HIP kernels.

For each of the 256 classes [ab|cd] (a, b, c, d in s, p, d, f) it writes one
kernel that computes contracted Cartesian ERIs by

  * the Boys function F_m(T) of each primitive quartet,
  * the Obara-Saika vertical recurrence (VRR) for [e0|f0]^(m), with e on the
    bra and f on the ket, |e| in [La, La+Lb] and |f| in [Lc, Lc+Ld],
  * accumulation of the primitive quartets (contraction) in FP64,
  * the Head-Gordon-Pople horizontal recurrence (HRR), written in its
    closed binomial form (b on A, d on C),
  * the paper's compression (eqs. 9-10): per quartet b_max, eps, n-bit codes.

The paper itself computes with Rys quadrature (its section II-C); the
recurrences here are the Obara-Saika / Head-Gordon-Pople ones it cites as the
other family, chosen because they contract before the HRR.

Two work mappings are emitted:

  mode T  one lane computes one contracted quartet; every intermediate is a
          named register value of straight-line code.
  mode W  one group of lanes ("slot") computes one quartet: lane l owns one
          bra index e of [e0|..] (two when a slot would exceed 64 lanes,
          split by the parity of |e|).  Each lane builds [e0|00]^(m) along
          its own z->y->x path, then the ket recurrence for all f in
          registers; the one term of the ket VRR that couples different e,
          [e-1_i 0|f0]^(m+1), is fetched from the owning lane by a wave
          permute.  After contraction, each lane applies the ket HRR to its
          own e, the results go through LDS, and lanes owning ket indices cd
          apply the bra HRR, reduce b_max and quantise.
"""
import itertools
import math
import os

REALS = {"fp64": "double", "mixed": "float", "rys": "double", "rys32": "float"}

# kernel name -> 1 if its packed-stream path stages codes in dynamic LDS (sized
# at launch), 0 if in the kernel's own LDS once the HRR staging is consumed
PACK_DYNAMIC_LDS = {}


# ---------------------------------------------------------------------------
# Cartesian bookkeeping
# ---------------------------------------------------------------------------
def ncart(L):
    return (L + 1) * (L + 2) // 2


def comps(L):
    return [(lx, ly, L - lx - ly) for lx in range(L, -1, -1) for ly in range(L - lx, -1, -1)]


def cidx(c):
    L = sum(c)
    lx, ly = c[0], c[1]
    return (L - lx) * (L - lx + 1) // 2 + (L - lx - ly)


def vadd(a, b):
    return (a[0] + b[0], a[1] + b[1], a[2] + b[2])


def vsub(a, b):
    return (a[0] - b[0], a[1] - b[1], a[2] - b[2])


UNIT = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
ZERO = (0, 0, 0)


def lower_dir(v, rule):
    nz = [i for i in range(3) if v[i] > 0]
    if rule == "first":
        return nz[0]
    if rule == "last":
        return nz[-1]
    # largest component, first on ties
    return max(nz, key=lambda i: (v[i], -i))


def class_id(la, lb, lc, ld):
    return la * 64 + lb * 16 + lc * 4 + ld


def class_id5(la, lb, lc, ld):
    """Index of a class in the kernel table (angular momenta up to 4)."""
    return la * 125 + lb * 25 + lc * 5 + ld


def kernel_name(prec, user, alt=False):
    """eri_<prec>_cNNN for s-f classes (NNN = La*64+Lb*16+Lc*4+Ld), eri_<prec>_gNNN
    (NNN = La*125+Lb*25+Lc*5+Ld) for classes with a g shell (derivative shells);
    suffix _a for the alternate-mode kernel of a class."""
    suf = "_a" if alt else ""
    if max(user) <= 3:
        return "eri_%s_c%03d%s" % (prec, class_id(*user), suf)
    return "eri_%s_g%03d%s" % (prec, class_id5(*user), suf)


# classes with one g shell and s, p, d on the others: the exponent derivatives
# of d shells (L + 2) in the adjoint
MAXVAR = 8   # launch variants per class (ERI_MAXVAR)

G_CLASSES = [c for c in itertools.product(range(5), repeat=4) if sorted(c)[-1] == 4 and sorted(c)[-2] <= 2]


def class_of(cid):
    return (cid >> 6) & 3, (cid >> 4) & 3, (cid >> 2) & 3, cid & 3


# ---------------------------------------------------------------------------
# Class plan: orientation, mode and the VRR element sets
# ---------------------------------------------------------------------------
class ClassPlan:
    """Orientation, work mapping and VRR element set of one class.

    `perm` maps computed shells to user shells: the kernel computes
    [s_perm0 s_perm1 | s_perm2 s_perm3].  Within each pair the shell with the
    larger L goes first, so the HRR always moves the smaller angular momentum
    (the canonical ordering of eq. 4); this keeps the HRR short and, with
    far-apart centres and mixed tight/diffuse exponents, avoids the loss of
    digits of transferring a high L across a long bond.  The bra/ket order is
    chosen for the register footprint of mode W."""

    def __init__(self, la, lb, lc, ld, mode=None, perm=None):
        self.user = (la, lb, lc, ld)
        self.cid = class_id(la, lb, lc, ld)
        if perm is None:
            perm = self._choose_perm()
        self.perm = tuple(perm)
        a, b, c, d = (self.user[k] for k in self.perm)
        self.a, self.b, self.c, self.d = a, b, c, d
        self.Lab, self.Lcd, self.Ltot = a + b, c + d, a + b + c + d
        self.E_T = [e for L in range(a, a + b + 1) for e in comps(L)]
        self.F_T = [f for L in range(c, c + d + 1) for f in comps(L)]
        self.n_eriq = ncart(la) * ncart(lb) * ncart(lc) * ncart(ld)
        self.rule = self._best_rule()
        self.elems = self._closure(self.rule)
        if mode is None:
            mode = self._choose_mode()
        self.mode = mode

    @property
    def swap(self):
        return self.perm[0] >= 2

    # ---- orientation ----------------------------------------------------
    def _choose_perm(self):
        la, lb, lc, ld = self.user
        bra = (0, 1) if la >= lb else (1, 0)
        ket = (2, 3) if lc >= ld else (3, 2)

        def est(lab, lc_, lcd):
            n_e = (lab + 1) * (lab + 2) * (lab + 3) // 6
            S = 1 if n_e <= 64 else 2
            lv = [ncart(k) * (lcd - k + 1) for k in range(lcd + 1)]
            live = max(sum(lv[max(0, k - 2):k + 1]) for k in range(len(lv)))
            return S * (live + sum(ncart(x) for x in range(lc_, lcd + 1)))

        keep = est(la + lb, max(lc, ld), lc + ld)
        swap = est(lc + ld, max(la, lb), la + lb)
        if swap < keep or (swap == keep and (lc + ld) > (la + lb)):
            return ket + bra
        return bra + ket

    # ---- VRR closure (mode T program) ------------------------------------
    def _closure(self, rule):
        need = {}
        stack = [(e, f, 0) for e in self.E_T for f in self.F_T]
        while stack:
            el = stack.pop()
            if el in need:
                continue
            e, f, m = el
            srcs = []
            if f != ZERO:
                i = lower_dir(f, rule)
                fp = vsub(f, UNIT[i])
                srcs += [(e, fp, m), (e, fp, m + 1)]
                if fp[i] >= 1:
                    fpp = vsub(fp, UNIT[i])
                    srcs += [(e, fpp, m), (e, fpp, m + 1)]
                if e[i] >= 1:
                    srcs.append((vsub(e, UNIT[i]), fp, m + 1))
                need[el] = ("ket", i)
            elif e != ZERO:
                i = lower_dir(e, rule)
                ep = vsub(e, UNIT[i])
                srcs += [(ep, ZERO, m), (ep, ZERO, m + 1)]
                if ep[i] >= 1:
                    epp = vsub(ep, UNIT[i])
                    srcs += [(epp, ZERO, m), (epp, ZERO, m + 1)]
                need[el] = ("bra", i)
            else:
                need[el] = ("base", None)
            stack.extend(srcs)
        return need

    def _best_rule(self):
        best = None
        for rule in ("first", "max", "last"):
            n = len(self._closure(rule))
            if best is None or n < best[0]:
                best = (n, rule)
        return best[1]

    # ---- mode choice -------------------------------------------------------
    def ket_live_estimate(self):
        # doubles live per lane in mode W: three consecutive ket levels + accumulators
        lv = [ncart(k) * (self.Lcd - k + 1) for k in range(self.Lcd + 1)]
        live = max(sum(lv[max(0, k - 2):k + 1]) for k in range(len(lv)))
        return live + len(self.F_T)

    def _choose_mode(self):
        n_elem = len(self.elems)
        regs_T = n_elem + len(self.E_T) * len(self.F_T) + self.n_eriq
        if n_elem <= 120 and self.n_eriq <= 64 and regs_T <= 240:
            return "T"
        return "W"

    # ---- algorithmic flop count -------------------------------------------
    def flops(self):
        """(per primitive quartet, per contracted quartet) algorithmic FLOPs:
        FMA = 2, add/mul = 1, div/sqrt/exp = 1; the VRR closure, Boys (table
        Taylor + recursion), setup and accumulation per primitive quartet; the
        recursive HGP HRR and the quantiser per quartet."""
        vrr = 0
        for (e, f, m), (kind, i) in self.elems.items():
            if kind == "base":
                vrr += 1
            elif kind == "bra":
                ep = vsub(e, UNIT[i])
                vrr += 3 + (3 if ep[i] >= 1 else 0)
            else:
                fp = vsub(f, UNIT[i])
                vrr += 3 + (3 if fp[i] >= 1 else 0) + (2 if e[i] >= 1 else 0)
        setup = 30
        boys = 30 + 3 * self.Ltot
        acc = len(self.E_T) * len(self.F_T)
        per_pq = setup + boys + vrr + acc
        # recursive HRR: bra (a, b+1) = (a+1, b) + AB (a, b) over all f, then ket
        a, b, c, d = self.a, self.b, self.c, self.d
        hb = 0
        for lb_ in range(1, b + 1):
            hb += ncart(lb_) * sum(ncart(x) for x in range(a, a + b - lb_ + 1))
        hb *= len(self.F_T)
        hk = 0
        for ld_ in range(1, d + 1):
            hk += ncart(ld_) * sum(ncart(x) for x in range(c, c + d - ld_ + 1))
        hk *= ncart(a) * ncart(b)
        per_q = 2 * (hb + hk) + 3 * self.n_eriq
        return per_pq, per_q


# ---------------------------------------------------------------------------
# Small code-emission helpers
# ---------------------------------------------------------------------------
class Emitter:
    def __init__(self):
        self.lines = []
        self.ind = 0

    def __call__(self, s=""):
        self.lines.append("    " * self.ind + s)

    def block(self, head):
        self(head + " {")
        self.ind += 1

    def end(self, tail=""):
        self.ind -= 1
        self("}" + tail)

    def text(self):
        return "\n".join(self.lines) + "\n"


def lit(x):
    return repr(float(x))


def binom(n, k):
    return math.comb(n, k)


def hrr_terms(b):
    """(k, coef, powers) of (a, b| = sum_k C(b,k) (AB)^(b-k) (a+k, 0|."""
    out = []
    for kx in range(b[0] + 1):
        for ky in range(b[1] + 1):
            for kz in range(b[2] + 1):
                coef = binom(b[0], kx) * binom(b[1], ky) * binom(b[2], kz)
                out.append(((kx, ky, kz), coef, (b[0] - kx, b[1] - ky, b[2] - kz)))
    return out


def mono_name(prefix, pw):
    if pw == ZERO:
        return None
    return "%s_%d%d%d" % (prefix, pw[0], pw[1], pw[2])


def emit_hrr_coefs(em, prefix, base, bs, real):
    """Declare the HRR coefficients C(b,k) (base)^(b-k) needed by the shells'
    components `bs`, each as one named constant, so every use of a
    coefficient reads the same bits."""
    need = set()
    for bb in bs:
        for (_, coef, pw) in hrr_terms(bb):
            if pw != ZERO:
                need.add((coef, pw))
    axis_max = [max([pw[i] for (_, pw) in need] + [0]) for i in range(3)]
    for i, ax in enumerate("xyz"):
        for k in range(1, axis_max[i] + 1):
            if k == 1:
                em("const %s %s_%s1 = (%s)%s[%d];" % (real, prefix, ax, real, base, i))
            else:
                em("const %s %s_%s%d = %s_%s%d * %s_%s1;" % (real, prefix, ax, k, prefix, ax, k - 1, prefix, ax))
    for coef, pw in sorted(need):
        parts = ["%s_%s%d" % (prefix, "xyz"[i], pw[i]) for i in range(3) if pw[i] > 0]
        if coef != 1:
            parts = ["(%s)%s" % (real, lit(coef))] + parts
        em("const %s %s = %s;" % (real, coef_name(prefix, coef, pw), " * ".join(parts)))


def coef_name(prefix, coef, pw):
    return "%s_k%d_%d%d%d" % (prefix, coef, pw[0], pw[1], pw[2])


def hrr_expr(b, a, getter, prefix):
    """Closed-form HRR of (a, b| = sum_k C(b,k) (AB)^(b-k) (a+k, 0| from values
    getter(a + k), as an explicit fma chain (evaluation order fixed)."""
    terms = hrr_terms(b)
    expr = None
    for k, coef, pw in terms:
        if pw == ZERO:
            expr = getter(vadd(a, k))
    for k, coef, pw in terms:
        if pw == ZERO:
            continue
        expr = "fma(%s, %s, %s)" % (coef_name(prefix, coef, pw), getter(vadd(a, k)), expr)
    return expr


# ---------------------------------------------------------------------------
# Mode T kernel
# ---------------------------------------------------------------------------
def emit_mode_T(cp, prec, name):
    real = REALS[prec]
    mixed = prec == "mixed"
    em = Emitter()
    a, b, c, d = cp.a, cp.b, cp.c, cp.d
    em("// class [%d%d|%d%d] computed as shells %s = [%d%d|%d%d], mode T, %s" % (cp.user + (cp.perm, a, b, c, d, prec)))
    em("__global__ __launch_bounds__(256) void %s(eri_class_args A)" % name)
    em.block("")
    em("const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;")
    em("if (t >= A.n_items) return;")
    em("const eri_item it = A.items[t];")
    em("const bool sb = it.bra < 0, sk = it.ket < 0;   // pair stored in swapped order")
    em("const eri_shell_pair BP = A.pairs[it.bra & 0x7fffffff];")
    em("const eri_shell_pair KP = A.pairs[it.ket & 0x7fffffff];")
    # accumulators
    acc = {}
    for e in cp.E_T:
        for f in cp.F_T:
            acc[(e, f)] = "acc_%d_%d_%d__%d_%d_%d" % (e + f)
            em("double %s = 0.0;" % acc[(e, f)])
    em.block("for (int ib = 0; ib < BP.nprim; ++ib)")
    em("const eri_prim_pair B = A.prims[BP.prim_off + ib];")
    em.block("for (int ik = 0; ik < KP.nprim; ++ik)")
    em("const eri_prim_pair K = A.prims[KP.prim_off + ik];")
    em("eri_pq_fp64 S;")
    em("eri_pq_setup(B, K, S);")
    em("double F[%d];" % (cp.Ltot + 1))
    em("eri_boys<%d>(S.T, F);" % cp.Ltot)
    # coefficients in the working type
    em("const %s PAx = (%s)B.PA[0], PAy = (%s)B.PA[1], PAz = (%s)B.PA[2];" % ((real,) * 4))
    em("const %s QCx = (%s)K.PA[0], QCy = (%s)K.PA[1], QCz = (%s)K.PA[2];" % ((real,) * 4))
    em("const %s WPx = (%s)S.WP[0], WPy = (%s)S.WP[1], WPz = (%s)S.WP[2];" % ((real,) * 4))
    em("const %s WQx = (%s)S.WQ[0], WQy = (%s)S.WQ[1], WQz = (%s)S.WQ[2];" % ((real,) * 4))
    em("const %s hp = (%s)B.hp, hq = (%s)K.hp, hpq = (%s)S.hpq, rp = (%s)S.rho_p, rq = (%s)S.rho_q;" % ((real,) * 6))
    names = {}
    order = sorted(cp.elems.keys(), key=lambda el: (sum(el[1]), sum(el[0]), el[0], el[1], -el[2]))
    n = 0
    for el in order:
        names[el] = "v%d" % n
        n += 1
    for el in order:
        e, f, m = el
        kind, i = cp.elems[el]
        ax = "xyz"[i] if i is not None else None
        if kind == "base":
            expr = "(%s)(S.pref * F[%d])" % (real, m)
        elif kind == "bra":
            ep = vsub(e, UNIT[i])
            expr = "PA%s * %s + WP%s * %s" % (ax, names[(ep, ZERO, m)], ax, names[(ep, ZERO, m + 1)])
            if ep[i] >= 1:
                epp = vsub(ep, UNIT[i])
                expr += " + (%s * hp) * (%s - rp * %s)" % (lit(ep[i]), names[(epp, ZERO, m)], names[(epp, ZERO, m + 1)])
        else:
            fp = vsub(f, UNIT[i])
            expr = "QC%s * %s + WQ%s * %s" % (ax, names[(e, fp, m)], ax, names[(e, fp, m + 1)])
            if fp[i] >= 1:
                fpp = vsub(fp, UNIT[i])
                expr += " + (%s * hq) * (%s - rq * %s)" % (lit(fp[i]), names[(e, fpp, m)], names[(e, fpp, m + 1)])
            if e[i] >= 1:
                expr += " + (%s * hpq) * %s" % (lit(e[i]), names[(vsub(e, UNIT[i]), fp, m + 1)])
        em("const %s %s = %s;" % (real, names[el], expr))
    for e in cp.E_T:
        for f in cp.F_T:
            if mixed:
                em("%s += (double)%s;" % (acc[(e, f)], names[(e, f, 0)]))
            else:
                em("%s += %s;" % (acc[(e, f)], names[(e, f, 0)]))
    em.end()
    em.end()
    # HRR: ket first over every target e, then bra
    ca, cb, cc, cd = comps(a), comps(b), comps(c), comps(d)
    emit_hrr_coefs(em, "ab", "BP.AB", cb, real)
    emit_hrr_coefs(em, "cd", "KP.AB", cd, real)
    y = {}
    for e in cp.E_T:
        for ci in cc:
            for di in cd:
                nm = "y_%d%d%d_%d%d%d_%d%d%d" % (e + ci + di)
                y[(e, ci, di)] = nm
                expr = hrr_expr(di, ci, lambda f, e=e: "(%s)%s" % (real, acc[(e, f)]), "cd")
                em("const %s %s = %s;" % (real, nm, expr))
    outs = []
    for ia, ai in enumerate(ca):
        for ib_, bi in enumerate(cb):
            for ic, ci in enumerate(cc):
                for id_, di in enumerate(cd):
                    nm = "o%d" % len(outs)
                    expr = hrr_expr(bi, ai, lambda e, ci=ci, di=di: y[(e, ci, di)], "ab")
                    em("const double %s = (double)(%s);" % (nm, expr))
                    outs.append((nm, (ia, ib_, ic, id_)))
    emit_store_T(em, cp, outs, prec)
    em.end()
    return name, em.text()


RYS_LMAX = 4      # classes with L_tot <= 4: one lane per quartet (at most 3 roots); larger: a workgroup
RYS_DEG = 8       # degree of the Chebyshev series of the Rys rule (gen_rys_table.DEG)


def emit_mode_R(cp, name, real="double"):
    """Rys-quadrature kernel of a class (Sec. II-C, eqs. 5-8), one lane per
    quartet, in the orientation cp.perm of the Obara-Saika kernels.  With
    real = "float" the recurrences, transfers and the node sum run in FP32
    (the paper's single-precision Rys stages): the rule, the setup and the
    prefactor stay FP64, G(0, 0) of z carries the weight only, and each
    primitive quartet's FP32 node sum is scaled by the FP64 prefactor into the
    FP64 contraction sums.
    Per primitive quartet the n = L_tot/2 + 1 nodes x_r = t_r^2 and weights
    w_r of the Rys rule at T come from the tabulated fits (eri_rys_rule);
    per node and axis the 2D integrals G(n, m), n <= L_a + L_b, m <= L_c + L_d,
    follow the Rys recurrences
        G(n+1, 0) = C00 G(n, 0) + n B10 G(n-1, 0)
        G(n, m+1) = C00' G(n, m) + m B01 G(n, m-1) + n B00 G(n-1, m)
    with B00 = x/(2(p+q)), B10 = (1 - q x/(p+q))/(2p), B01 = (1 - p x/(p+q))/(2q),
    C00 = (P-A) + x (W-P), C00' = (Q-C) + x (W-Q), G(0, 0) = 1 for x and y and
    the weight times the prefactor for z; the horizontal transfer moves
    angular momentum to B and D per axis (I(a, b+1) = I(a+1, b) + (A-B) I(a,
    b)); each ERI adds sum_r Ix Iy Iz.  Returns (name, source, FLOPs per
    primitive quartet)."""
    a, b, c, d = cp.a, cp.b, cp.c, cp.d
    Lab, Lcd = a + b, c + d
    N = cp.Ltot // 2 + 1
    em = Emitter()
    flops = [30 + 2 * N * 3 * RYS_DEG + 4 * N]      # setup, the node/weight series, their scaling

    def count(expr):
        flops[0] += expr.count("*") + expr.count(" + ") + expr.count(" - ")
    em("// class [%d%d|%d%d] computed as shells %s = [%d%d|%d%d], Rys quadrature (%d nodes), one lane per quartet"
       % (cp.user + (cp.perm, a, b, c, d, N)))
    em("__global__ __launch_bounds__(256) void %s(eri_class_args A)" % name)
    em.block("")
    em("const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;")
    em("if (t >= A.n_items) return;")
    em("const eri_item it = A.items[t];")
    em("const bool sb = it.bra < 0, sk = it.ket < 0;   // pair stored in swapped order")
    em("const eri_shell_pair BP = A.pairs[it.bra & 0x7fffffff];")
    em("const eri_shell_pair KP = A.pairs[it.ket & 0x7fffffff];")
    ca, cb, cc, cd = comps(a), comps(b), comps(c), comps(d)
    outs = []
    for ia, ai in enumerate(ca):
        for ib_, bi in enumerate(cb):
            for ic, ci in enumerate(cc):
                for id_, di in enumerate(cd):
                    outs.append(("o%d" % len(outs), (ia, ib_, ic, id_), (ai, bi, ci, di)))
    for nm, _, _ in outs:
        em("double %s = 0.0;" % nm)
    em.block("for (int ib = 0; ib < BP.nprim; ++ib)")
    em("const eri_prim_pair B = A.prims[BP.prim_off + ib];")
    em.block("for (int ik = 0; ik < KP.nprim; ++ik)")
    em("const eri_prim_pair K = A.prims[KP.prim_off + ik];")
    em("eri_pq_fp64 S;")
    em("eri_pq_setup(B, K, S);")
    em("double rx[%d], rw[%d];" % (N, N))
    em("eri_rys_rule<%d>(S.T, rx, rw);" % N)
    f32 = real == "float"

    def rl(x):
        return lit(x) + ("f" if f32 else "")
    if f32:
        for nm, _, _ in outs:
            em("float t%s = 0.0f;" % nm)
    em("#pragma unroll")
    em.block("for (int r = 0; r < %d; ++r)" % N)
    em("const double u = rx[r];")
    em("const %s B00 = (%s)(u * S.hpq);" % (real, real))
    em("const %s B10 = (%s)(B.hp - B.hp * S.rho_p * u);" % (real, real))
    em("const %s B01 = (%s)(K.hp - K.hp * S.rho_q * u);" % (real, real))
    flops[0] += 5
    defined = set()

    def g(ax, n, m):
        nm = "g%s_%d_%d" % (ax, n, m)
        if nm in defined:
            return nm
        i = "xyz".index(ax)
        if n == 0 and m == 0:
            if f32:
                expr = "(float)rw[r]" if ax == "z" else "1.0f"
            else:
                expr = "rw[r] * S.pref" if ax == "z" else "1.0"
        elif m == 0:
            expr = "C0%s * %s" % (ax, g(ax, n - 1, 0))
            if n - 1 >= 1:
                expr += " + %s * B10 * %s" % (rl(n - 1), g(ax, n - 2, 0))
        else:
            expr = "D0%s * %s" % (ax, g(ax, n, m - 1))
            if m - 1 >= 1:
                expr += " + %s * B01 * %s" % (rl(m - 1), g(ax, n, m - 2))
            if n >= 1:
                expr += " + %s * B00 * %s" % (rl(n), g(ax, n - 1, m - 1))
        em("const %s %s = %s;" % (real, nm, expr))
        count(expr)
        defined.add(nm)
        return nm

    def kh(ax, n, cx, dx):
        # ket transfer: K(n, c, d+1) = K(n, c+1, d) + (C-D) K(n, c, d); K(n, c, 0) = G(n, c)
        if dx == 0:
            return g(ax, n, cx)
        nm = "k%s_%d_%d_%d" % (ax, n, cx, dx)
        if nm in defined:
            return nm
        expr = "%s + CD%s * %s" % (kh(ax, n, cx + 1, dx - 1), ax, kh(ax, n, cx, dx - 1))
        em("const %s %s = %s;" % (real, nm, expr))
        count(expr)
        defined.add(nm)
        return nm

    def ih(ax, ax_a, bx, cx, dx):
        # bra transfer: I(a, b+1) = I(a+1, b) + (A-B) I(a, b); I(a, 0) = K(a)
        if bx == 0:
            return kh(ax, ax_a, cx, dx)
        nm = "i%s_%d_%d_%d_%d" % (ax, ax_a, bx, cx, dx)
        if nm in defined:
            return nm
        expr = "%s + AB%s * %s" % (ih(ax, ax_a + 1, bx - 1, cx, dx), ax, ih(ax, ax_a, bx - 1, cx, dx))
        em("const %s %s = %s;" % (real, nm, expr))
        count(expr)
        defined.add(nm)
        return nm
    for i, ax in enumerate("xyz"):
        em("const %s C0%s = (%s)(B.PA[%d] + u * S.WP[%d]);" % (real, ax, real, i, i))
        em("const %s D0%s = (%s)(K.PA[%d] + u * S.WQ[%d]);" % (real, ax, real, i, i))
        em("const %s AB%s = (%s)BP.AB[%d], CD%s = (%s)KP.AB[%d];" % (real, ax, real, i, ax, real, i))
        flops[0] += 4
    for nm, _, (ai, bi, ci, di) in outs:
        fx = ih("x", ai[0], bi[0], ci[0], di[0])
        fy = ih("y", ai[1], bi[1], ci[1], di[1])
        fz = ih("z", ai[2], bi[2], ci[2], di[2])
        em("%s += %s * %s * %s;" % (("t" + nm) if f32 else nm, fx, fy, fz))
        flops[0] += 3
    em.end()
    if f32:
        for nm, _, _ in outs:
            em("%s = fma((double)t%s, S.pref, %s);" % (nm, nm, nm))
        flops[0] += 2 * len(outs)
    em.end()
    em.end()
    emit_store_T(em, cp, [(nm, ix) for nm, ix, _ in outs], "rys")
    em.end()
    return name, em.text(), flops[0]


RYSW_LDS = 44 * 1024   # LDS of the 1D-integral buffer of one workgroup-per-quartet Rys kernel
# launch variants of those kernels:
# (name suffix, LDS budget of the buffer, waves per SIMD, thread scale, node loop unrolled, tag)
RYSW_VARIANTS = (("", RYSW_LDS, 1, 1, True, 0), ("_b", 100 * 1024, 1, 1, True, 7), ("_o2", RYSW_LDS, 2, 1, True, 2),
                 ("_w", RYSW_LDS, 4, 2, True, 8), ("_wo2", RYSW_LDS, 2, 2, True, 9),
                 ("_n", RYSW_LDS, 1, 1, False, 10), ("_no2", RYSW_LDS, 2, 1, False, 11),
                 ("_nwo2", RYSW_LDS, 2, 2, False, 12))


def rysw_shape(cp, lds_budget=RYSW_LDS, vbytes=8, nt_scale=1):
    """(threads, ERIs per thread, primitive quartets per batch, 1D values
    per node and axis) of the workgroup-per-quartet Rys kernel of a class
    (1D values of vbytes bytes)."""
    n = cp.n_eriq
    NT = nt_scale * (256 if n > 1024 else 128 if n > 256 else 64)
    N = cp.Ltot // 2 + 1
    NI = (cp.a + 1) * (cp.b + 1) * (cp.c + 1) * (cp.d + 1)
    NB = max(1, min(NT // (3 * N), lds_budget // (3 * N * NI * vbytes)))
    return NT, (n + NT - 1) // NT, NB, NI


def emit_mode_RW(cp, name, lds_budget=RYSW_LDS, occupancy=1, real="double", nt_scale=1, unroll=True):
    """Rys-quadrature kernel of a class whose ERIs do not fit one lane (Sec.
    II-C, eqs. 5-8): one workgroup per quartet, in the orientation cp.perm.
    Per batch of NB primitive quartets:
      1. one lane per primitive quartet and entry of the n-point Rys rule
         at T (eri_rys_rule_entry: one node or weight), plus the
         Gaussian-product setup, into LDS;
      2. one lane per (primitive quartet, node, axis): the 2D integrals
         G(n, m) of the Rys recurrences
             G(n+1, 0) = C00 G(n, 0) + n B10 G(n-1, 0)
             G(n, m+1) = C00' G(n, m) + m B01 G(n, m-1) + n B00 G(n-1, m),
         then the transfers to B (I(a, b+1) = I(a+1, b) + (A-B) I(a, b)) and
         to D, giving every 1D factor I(a', b', c', d') of that node and
         axis, into LDS (the weight and prefactor ride on the z factors);
      3. each thread owns ERIs k = thread + NT s of the computed layout and
         adds sum over nodes of Ix Iy Iz, the three factors read from LDS at
         offsets packed per ERI in a table.
    Then b_max over the workgroup, and the store / quantise / pack of the
    other kernels.  With real = "float" the recurrences, transfers, 1D
    factors and the node sum are FP32 (the paper's single-precision Rys
    stages); the rule, the setup and the prefactor stay FP64, the z factors
    carry the weight only, and each primitive quartet's FP32 node sum is
    scaled by the FP64 prefactor into FP64 contraction sums.  Returns (name,
    source, FLOPs per primitive quartet)."""
    a, b, c, d = cp.a, cp.b, cp.c, cp.d
    n = cp.n_eriq
    f32 = real == "float"
    vb = 4 if f32 else 8
    NT, S, NB, NI = rysw_shape(cp, lds_budget, vb, nt_scale)
    N = cp.Ltot // 2 + 1
    NQ = 2 * N + 18
    nbuf = NB * N * 3 * NI
    nbuf = max(nbuf, (4 * n + vb - 1) // vb)      # the packed path stages int32 codes over it

    def rl(x):
        return lit(x) + ("f" if f32 else "")
    dims = (a + 1, b + 1, c + 1, d + 1)

    def idx1(t):
        return ((t[0] * dims[1] + t[1]) * dims[2] + t[2]) * dims[3] + t[3]
    ca, cb, cc, cd = comps(a), comps(b), comps(c), comps(d)
    tab = []
    for ai in ca:
        for bi in cb:
            for ci in cc:
                for di in cd:
                    ox, oy, oz = [idx1((ai[x], bi[x], ci[x], di[x])) + x * NI for x in range(3)]
                    tab.append(ox | (oy << 10) | (oz << 20))
    assert 3 * NI <= 1024 and len(tab) == n
    em = Emitter()
    flops = [30 + 2 * N * 3 * RYS_DEG + 2 * N]    # setup, the node/weight series, the weights' prefactor

    def count(expr):
        # one (node, axis) task: every node and axis of a primitive quartet runs it
        flops[0] += 3 * N * (expr.count("*") + expr.count(" + ") + expr.count(" - "))
    em("// class [%d%d|%d%d] computed as shells %s = [%d%d|%d%d], Rys quadrature (%d nodes), one workgroup of %d "
       "threads per quartet" % (cp.user + (cp.perm, a, b, c, d, N, NT)))
    em("static __device__ const uint32_t %s_tab[%d] = {" % (name, n))
    for i in range(0, n, 12):
        em("    " + ", ".join(str(v) for v in tab[i:i + 12]) + ",")
    em("};")
    if occupancy > 1:
        em("__global__ __launch_bounds__(%d, %d) void %s(eri_class_args A)" % (NT, occupancy, name))
    else:
        em("__global__ __launch_bounds__(%d) void %s(eri_class_args A)" % (NT, name))
    em.block("")
    em("__shared__ %s s_I[%d];   // [batch][node][axis][1D index]" % (real, nbuf))
    em("__shared__ double s_q[%d];   // per primitive quartet: nodes, weights, C00/C00' parts, B parts" % (NB * NQ))
    em("__shared__ double s_red[%d];" % (NT // 64))
    em("const int tid = threadIdx.x;")
    em("const int64_t qi = blockIdx.x;")
    em("if (qi >= A.n_items) return;   // uniform over the workgroup")
    em("const eri_item it = A.items[qi];")
    em("const bool sb = it.bra < 0, sk = it.ket < 0;   // pair stored in swapped order")
    em("const eri_shell_pair BP = A.pairs[it.bra & 0x7fffffff];")
    em("const eri_shell_pair KP = A.pairs[it.ket & 0x7fffffff];")
    em("const int nket = KP.nprim;")
    em("const int npq = BP.nprim * nket;")
    em("uint32_t off[%d];" % S)
    em("double acc[%d];" % S)
    em("#pragma unroll")
    em.block("for (int s = 0; s < %d; ++s)" % S)
    em("const int k = tid + %d * s;" % NT)
    em("off[s] = k < %d ? %s_tab[k] : 0u;" % (n, name))
    em("acc[s] = 0.0;")
    em.end()
    em.block("for (int j0 = 0; j0 < npq; j0 += %d)" % NB)
    em("__syncthreads();   // the previous batch's factors are consumed")
    em("const int nb = min(%d, npq - j0);" % NB)
    em.block("for (int t = tid; t < nb * %d; t += %d)" % (2 * N, NT))
    em("const int jb = t / %d, e = t - jb * %d;" % (2 * N, 2 * N))
    em("const int j = j0 + jb;")
    em("const int ib = j / nket, ik = j - ib * nket;")
    em("const eri_prim_pair B = A.prims[BP.prim_off + ib];")
    em("const eri_prim_pair K = A.prims[KP.prim_off + ik];")
    em("eri_pq_fp64 S;")
    em("eri_pq_setup(B, K, S);")
    em("const double v = eri_rys_rule_entry<%d>(S.T, e);" % N)
    em("double* q = s_q + jb * %d;" % NQ)
    if f32:
        em("q[e] = v;")
    else:
        em("q[e] = e < %d ? v : v * S.pref;" % N)
    em.block("if (e == 0)")
    em("q[%d] = S.pref;" % (2 * N + 17))
    for i in range(3):
        em("q[%d] = B.PA[%d]; q[%d] = S.WP[%d]; q[%d] = K.PA[%d]; q[%d] = S.WQ[%d];"
           % (2 * N + i, i, 2 * N + 3 + i, i, 2 * N + 6 + i, i, 2 * N + 9 + i, i))
    em("q[%d] = S.hpq; q[%d] = B.hp; q[%d] = S.rho_p; q[%d] = K.hp; q[%d] = S.rho_q;"
       % tuple(2 * N + 12 + i for i in range(5)))
    em.end()
    em.end()
    em("__syncthreads();")
    em.block("for (int t = tid; t < nb * %d; t += %d)" % (3 * N, NT))
    em("const int jb = t / %d, rr = t - jb * %d;" % (3 * N, 3 * N))
    em("const int r = rr / 3, ax = rr - 3 * r;")
    em("const double* q = s_q + jb * %d;" % NQ)
    em("const double u = q[r];")
    R = real
    em("const %s B00 = (%s)(u * q[%d]);" % (R, R, 2 * N + 12))
    em("const %s B10 = (%s)(q[%d] - q[%d] * q[%d] * u);" % (R, R, 2 * N + 13, 2 * N + 13, 2 * N + 14))
    em("const %s B01 = (%s)(q[%d] - q[%d] * q[%d] * u);" % (R, R, 2 * N + 15, 2 * N + 15, 2 * N + 16))
    em("const %s C00 = (%s)(q[%d + ax] + u * q[%d + ax]);" % (R, R, 2 * N, 2 * N + 3))
    em("const %s D00 = (%s)(q[%d + ax] + u * q[%d + ax]);" % (R, R, 2 * N + 6, 2 * N + 9))
    em("const %s AB = (%s)(ax == 0 ? BP.AB[0] : ax == 1 ? BP.AB[1] : BP.AB[2]);" % (R, R))
    em("const %s CD = (%s)(ax == 0 ? KP.AB[0] : ax == 1 ? KP.AB[1] : KP.AB[2]);" % (R, R))
    em("const %s g_0_0 = ax == 2 ? (%s)q[%d + r] : %s;" % (R, R, N, rl(1)))
    flops[0] += N * (5 + 3 * 4)
    defined = {"g_0_0"}

    def g(nn, m):
        nm = "g_%d_%d" % (nn, m)
        if nm in defined:
            return nm
        if m == 0:
            expr = "C00 * %s" % g(nn - 1, 0)
            if nn - 1 >= 1:
                expr += " + %s * B10 * %s" % (rl(nn - 1), g(nn - 2, 0))
        else:
            expr = "D00 * %s" % g(nn, m - 1)
            if m - 1 >= 1:
                expr += " + %s * B01 * %s" % (rl(m - 1), g(nn, m - 2))
            if nn >= 1:
                expr += " + %s * B00 * %s" % (rl(nn), g(nn - 1, m - 1))
        em("const %s %s = %s;" % (real, nm, expr))
        count(expr)
        defined.add(nm)
        return nm

    def kh(nn, cx, dx):
        if dx == 0:
            return g(nn, cx)
        nm = "k_%d_%d_%d" % (nn, cx, dx)
        if nm in defined:
            return nm
        expr = "%s + CD * %s" % (kh(nn, cx + 1, dx - 1), kh(nn, cx, dx - 1))
        em("const %s %s = %s;" % (real, nm, expr))
        count(expr)
        defined.add(nm)
        return nm

    def ih(ax_a, bx, cx, dx):
        if bx == 0:
            return kh(ax_a, cx, dx)
        nm = "i_%d_%d_%d_%d" % (ax_a, bx, cx, dx)
        if nm in defined:
            return nm
        expr = "%s + AB * %s" % (ih(ax_a + 1, bx - 1, cx, dx), ih(ax_a, bx - 1, cx, dx))
        em("const %s %s = %s;" % (real, nm, expr))
        count(expr)
        defined.add(nm)
        return nm
    em("%s* I = s_I + ((jb * %d + r) * 3 + ax) * %d;" % (real, N, NI))
    # column by column of the ket (c', d'): its transfers to B, stored at once;
    # in the variants for the largest classes (node loop not unrolled) a
    # scheduling barrier between columns keeps the compiler from hoisting
    # every column's work (those ran out of registers); elsewhere it cost time
    for cdx in itertools.product(range(dims[2]), range(dims[3])):
        for abx in itertools.product(range(dims[0]), range(dims[1])):
            t = abx + cdx
            em("I[%d] = %s;" % (idx1(t), ih(*t)))
        if NI > 64 and not unroll:
            em("__builtin_amdgcn_sched_barrier(0);")
    em.end()
    em("__syncthreads();")
    em.block("for (int jb = 0; jb < nb; ++jb)")
    if f32:
        em("float t[%d];" % S)
        em("#pragma unroll")
        em("for (int s = 0; s < %d; ++s) t[s] = 0.0f;" % S)
    em("#pragma unroll" if unroll else "#pragma unroll 1")
    em.block("for (int r = 0; r < %d; ++r)" % N)
    em("const %s* I = s_I + (jb * %d + r) * %d;" % (real, N, 3 * NI))
    em("#pragma unroll")
    em("for (int s = 0; s < %d; ++s) %s = fma(I[off[s] & 1023u] * I[(off[s] >> 10) & 1023u], "
       "I[off[s] >> 20], %s);" % ((S,) + (("t[s]", "t[s]") if f32 else ("acc[s]", "acc[s]"))))
    em.end()
    if f32:
        em("const double pf = s_q[jb * %d + %d];" % (NQ, 2 * N + 17))
        em("#pragma unroll")
        em("for (int s = 0; s < %d; ++s) acc[s] = fma((double)t[s], pf, acc[s]);" % S)
        flops[0] += 2 * n
    em.end()
    em.end()
    flops[0] += 3 * N * n
    # epilogue: user-layout index of each owned ERI, b_max over the workgroup, stores
    emit_slot(em, "qi")
    em("const int64_t obase = oslot * %d;" % n)
    nc = [ncart(L) for L in (a, b, c, d)]
    em("int uix[%d];" % S)
    em("double bmax = 0.0;")
    em("#pragma unroll")
    em.block("for (int s = 0; s < %d; ++s)" % S)
    em("const int k = tid + %d * s;" % NT)
    em("const int id_ = k %% %d, ic = (k / %d) %% %d, ib = (k / %d) %% %d, ia = k / %d;"
       % (nc[3], nc[3], nc[2], nc[3] * nc[2], nc[1], nc[3] * nc[2] * nc[1]))
    st = user_strides(cp)
    bra = "ia * %d + ib * %d" % (st[0], st[1])
    if a == b and st[0] != st[1]:
        bra = "(sb ? ia * %d + ib * %d : %s)" % (st[1], st[0], bra)
    ket = "ic * %d + id_ * %d" % (st[2], st[3])
    if c == d and st[2] != st[3]:
        ket = "(sk ? ic * %d + id_ * %d : %s)" % (st[3], st[2], ket)
    em("uix[s] = %s + %s;" % (bra, ket))
    em("if (k < %d) bmax = fmax(bmax, fabs(acc[s]));" % n)
    em.end()
    em.block("if (A.out_eri)")
    em("#pragma unroll")
    em("for (int s = 0; s < %d; ++s) if (tid + %d * s < %d) A.out_eri[obase + uix[s]] = acc[s];" % (S, NT, n))
    em.end()
    em.block("if (A.out_codes)")
    em("for (int o = 32; o > 0; o >>= 1) bmax = fmax(bmax, __shfl_xor(bmax, o));")
    em("if ((tid & 63) == 0) s_red[tid >> 6] = bmax;")
    em("__syncthreads();")
    em("bmax = s_red[0];")
    em("#pragma unroll")
    em("for (int w = 1; w < %d; ++w) bmax = fmax(bmax, s_red[w]);" % (NT // 64))
    em("const double eps = bmax * A.cn;")
    em("const double inv = eri_inverse_scale(eps);")
    em("if (tid == 0 && A.out_scales) A.out_scales[oslot] = eps;")
    em.block("if (A.pack_bits)")
    em("const int wide = A.pack_bits > 16;")
    em("#pragma unroll")
    em("for (int s = 0; s < %d; ++s) if (tid + %d * s < %d) eri_stage_code(s_I, uix[s], wide, "
       "eri_quantize(acc[s], eps, inv, A.qmax));" % (S, NT, n))
    em("__syncthreads();")
    em("eri_pack_group(s_I, %d, 1, A.pack_bits, A.pack_per, (int)A.pack_wpq, "
       "reinterpret_cast<uint32_t*>(A.out_codes), gq, A.ring, tid, %d);" % (n, NT))
    em.end()
    em.block("else")
    em("#pragma unroll")
    em("for (int s = 0; s < %d; ++s) if (tid + %d * s < %d) eri_store_code(A.out_codes, obase + uix[s], "
       "A.code_bytes, eri_quantize(acc[s], eps, inv, A.qmax));" % (S, NT, n))
    em.end()
    em.end()
    em.end()
    return name, em.text(), flops[0]


def user_strides(cp):
    """Row-major strides of the user (a, b, c, d) layout, per computed shell."""
    n = [ncart(L) for L in cp.user]
    st = [n[1] * n[2] * n[3], n[2] * n[3], n[3], 1]
    return [st[k] for k in cp.perm]


def user_index(cp, ia, ib, ic, id_):
    """Row-major (a,b,c,d) index in the user orientation of computed indices."""
    st = user_strides(cp)
    return ia * st[0] + ib * st[1] + ic * st[2] + id_ * st[3]


def index_parts(cp, ia, ib, ic, id_):
    """C expressions of the bra and ket parts of the user-layout index of
    computed component indices; a pair of equal L may be stored swapped
    (flags sb, sk), which exchanges the strides of its two shells."""
    st = user_strides(cp)
    bn, bs = ia * st[0] + ib * st[1], ia * st[1] + ib * st[0]
    kn, ks = ic * st[2] + id_ * st[3], ic * st[3] + id_ * st[2]
    bra = "(sb ? %d : %d)" % (bs, bn) if (cp.a == cp.b and bs != bn) else str(bn)
    ket = "(sk ? %d : %d)" % (ks, kn) if (cp.c == cp.d and ks != kn) else str(kn)
    return bra, ket


def emit_slot(em, idx):
    """Output slot of launch item `idx`: class quartet qbase + idx in a ring."""
    em("const int64_t gq = A.qbase + %s;" % idx)
    em("const int64_t oslot = gq < A.ring ? gq : gq % A.ring;")


def emit_kx(em, cp):
    """kx: the user-layout offset of ket index kcd (computed (ic, id) =
    divmod(kcd, nd)); a ket pair of equal L stored swapped exchanges the
    strides of its two shells."""
    st = user_strides(cp)
    nd = ncart(cp.d)
    kn = "(int64_t)(kcd / %d) * %d + (int64_t)(kcd %% %d) * %d" % (nd, st[2], nd, st[3])
    if st[2] == nd * st[3] and st[3] == 1:
        kn = "(int64_t)kcd"
    if cp.c == cp.d and nd > 1:
        ks = "(int64_t)(kcd / %d) * %d + (int64_t)(kcd %% %d) * %d" % (nd, st[3], nd, st[2])
        em("const int64_t kx = sk ? %s : %s;" % (ks, kn))
    else:
        em("const int64_t kx = %s;" % kn)


def emit_pack_regs(em, cp, n, step, lane, guard, staged, ab_list, stage_base, coefs=None):
    """Codes of a single-chunk slot kernel's packed path: the bra HRR of every
    ket index this lane owns (j = lane, lane + step, ...) is quantised into
    registers (fast multiply-by-reciprocal quantiser unless some 1/eps of the
    workgroup overflows); after a barrier, when every lane has read the
    ket-HRR staging, the codes go over that staging in user order."""
    cb = comps(cp.b)
    NIT = (n + step - 1) // step
    em("int pkc[%d][%d];" % (NIT, len(ab_list)))
    for fast in (True, False):
        em.block("if (%s)" % ("!slow" if fast else "slow"))
        em("#pragma unroll")
        em.block("for (int it = 0; it < %d; ++it)" % NIT)
        em("const int j = %s + it * %d;" % (lane, step))
        em.block("if (%sj < %d)" % (guard, n))
        if coefs is not None:
            coefs()
        for k, (ai, bi) in enumerate(ab_list):
            expr = hrr_expr(bi, ai, staged, "ab")
            q = ("eri_quantize_mul((double)(%s), inv, A.qmax)" if fast else
                 "eri_quantize((double)(%s), eps, inv, A.qmax)") % expr
            em("pkc[it][%d] = %s;" % (k, q))
        em.end()
        em.end()
        em.end()
    em("__syncthreads();   // every lane has read the ket-HRR staging")
    em("#pragma unroll")
    em.block("for (int it = 0; it < %d; ++it)" % NIT)
    em("const int j = %s + it * %d;" % (lane, step))
    em.block("if (%sj < %d)" % (guard, n))
    em("const int kcd = j;")
    emit_kx(em, cp)
    emit_stage_codes(em, cp, len(ab_list), "s_u", stage_base, lambda k: "pkc[it][%d]" % k)
    em.end()
    em.end()


def emit_stage_codes(em, cp, nab, stage, stage_base, code):
    """Codes code(k) of bra index k at ket offset kx into the LDS staging
    (int32 when the uniform flag wide is set, else int16), one branch for
    all of them."""
    cb = comps(cp.b)
    for wide in (True, False):
        em.block("if (wide)" if wide else "else")
        t = "int32_t" if wide else "int16_t"
        for k in range(nab):
            ia_, ib_ = divmod(k, len(cb))
            bra, _ = index_parts(cp, ia_, ib_, 0, 0)
            em("reinterpret_cast<%s*>(%s)[%s(int)(%s + kx)] = (%s)%s;" % (t, stage, stage_base, bra, t, code(k)))
        em.end()


def narrow_chunking(NSU, nslot, NTE, NCD, n_eriq, NCH):
    """Chunks of the packed codes pass that leave room in s_u (NSU doubles)
    for the int16 codes of every slot: (chunk size, chunk count, byte
    offset of the codes), or None when that takes more than one chunk
    beyond twice the kernel's own."""
    code_dbl = (nslot * n_eriq * 2 + 7) // 8
    CHP = min(NCD, (NSU - code_dbl) // (nslot * NTE)) if NSU > code_dbl else 0
    if NCH == 1 or CHP < 1:
        return None
    NCHP = (NCD + CHP - 1) // CHP
    if NCHP > 2 * NCH + 1:
        return None
    return CHP, NCHP, nslot * NTE * CHP * 8


def narrow_arg(G, nar, CH):
    """emit_codes_pass's narrow argument for a kernel's chunk closures."""
    if not nar:
        return None
    CHP, NCHP, off = nar

    def enter():
        G["CH"], G["t"] = CHP, "s_tp"

    def leave():
        G["CH"], G["t"] = CH, "s_t"
    return NCHP, enter, leave, "(reinterpret_cast<unsigned char*>(s_u) + %d)" % off


def emit_codes_pass(em, NCH, ket_hrr_chunk, bra_hrr_chunk, slow_expr, pack_tail, narrow=None):
    """Second pass of a slot kernel: quantise and store.  The container width
    and whether any reciprocal 1/eps of the workgroup overflows are uniform
    over the workgroup, so they are decided once: the common case stores
    through a typed pointer with the multiply-by-reciprocal quantiser; the
    general case (eps so small that 1/eps overflows: codes from x / eps) keeps
    the generic store.  For a packed stream (A.pack_bits > 0, uniform) the
    codes are staged in LDS and pack_tail() writes the quartet's words.
    narrow = (chunk count, enter(), leave(), stage): with several chunks,
    int16 codes go over the kernel's own LDS behind smaller chunks (enter()
    and leave() switch the chunk closures), wider ones to dynamic LDS."""
    em.block("if (A.pack_bits)")
    em("const int wide = A.pack_bits > 16;")
    if NCH == 1:
        # single chunk: codes kept in registers (the accumulators are dead by
        # now) while every lane reads the ket-HRR staging, then written over
        # it and packed: no LDS beyond the kernel's own
        em("const int slow = %s;" % slow_expr)
        bra_hrr_chunk(0, 4)
        pack_tail("s_u")
    else:
        em("const int slow = %s;" % slow_expr)

        def staged(nch, stage):
            for fast in (True, False):
                em.block("if (!slow)" if fast else "else")
                for ch in range(nch):
                    ket_hrr_chunk(ch)
                    bra_hrr_chunk(ch, 3, "fast" if fast else "slow", stage=stage)
                em.end()
            pack_tail(stage)
        if narrow:
            nchp, enter, leave, stage = narrow
            em.block("if (!wide)")
            enter()
            staged(nchp, stage)
            leave()
            em.end()
            em.block("else")
            staged(NCH, "eri_pack_lds")
            em.end()
        else:
            staged(NCH, "eri_pack_lds")
    em.end()
    em.block("else")
    em("const int slow = %s;" % slow_expr)
    for i, (ct, nb) in enumerate((("int16_t", 2), ("int8_t", 1), ("int32_t", 4))):
        em.block("%s (!slow && A.code_bytes == %d)" % ("if" if i == 0 else "else if", nb))
        for ch in range(NCH):
            if NCH > 1:
                ket_hrr_chunk(ch)
            bra_hrr_chunk(ch, 2, ct)
        em.end()
    em.block("else")
    for ch in range(NCH):
        if NCH > 1:
            ket_hrr_chunk(ch)
        bra_hrr_chunk(ch, 2)
    em.end()
    em.end()


def adjoint_form(cp, prec):
    """Kernels that the adjoint launches: FP64 classes reached from user
    shells up to d by one derivative shift (L+1, L-1 or L+2 on one centre),
    so at most one shell above d."""
    return prec == "fp64" and sum(1 for l in cp.user if l > 2) <= 1


def emit_adj_T(em, outs):
    """Adjoint launch of a lane-per-quartet kernel: the lane's ERIs go into
    its quartet's gradient sums instead of the outputs."""
    em.block("if (A.adj.map)")
    em("eri_adj_quartet aq;")
    em("eri_adj_begin(A.adj, t, aq);")
    em("double g0 = 0.0, g1 = 0.0, g2 = 0.0;")
    for k, (nm, _) in enumerate(outs):
        em("eri_adj_add(A.adj, aq, i%d, %s, g0, g1, g2);" % (k, nm))
    em("eri_adj_finish(A.adj, t, aq, g0, g1, g2);")
    em("return;")
    em.end()


def emit_adj_slot(em, ket_hrr_chunk, bra_hrr_chunk, NCH, lane, ls, base, n, active, slot, nslot, off, room):
    """Adjoint launch of a slot or two-wavefront kernel (every thread of the
    workgroup takes it, so its barriers are uniform): the HRR outputs go into
    per-thread gradient sums, which the quartet's n threads add up through
    s_red; thread 0 of the quartet hands them to the gradients.  Each
    quartet's Gbar row is first copied into the free part of s_u (doubles
    off .. off + room, behind the HRR staging) when the workgroup's rows fit,
    so that the HRR outputs gather it from LDS."""
    em.block("if (A.adj.map)")
    em("eri_adj_quartet aq;")
    em("if (%s) eri_adj_begin(A.adj, qi, aq);" % active)
    em("double g0 = 0.0, g1 = 0.0, g2 = 0.0;")
    if room > 0:
        em("__syncthreads();   // the primitive staging in s_u is free")
        em.block("if (%d * A.adj.n_eriq <= %d)" % (nslot, room))
        em("double* s_g = s_u + %d + %s * A.adj.n_eriq;" % (off, slot))
        em("if (%s) for (int t = %s; t < A.adj.n_eriq; t += %d) s_g[t] = aq.g[t];" % (active, ls, n))
        em("if (%s) aq.g = s_g;" % active)
        em.end()
    for ch in range(NCH):
        ket_hrr_chunk(ch)
        bra_hrr_chunk(ch, 5)
    for v in ("g0", "g1", "g2"):
        em("__syncthreads();")
        em("s_red[%s] = %s;" % (lane, v))
        em("__syncthreads();")
        em.block("if (%s && %s == 0)" % (active, ls))
        em("double sum = 0.0;")
        em("for (int k = 0; k < %d; ++k) sum += s_red[%s + k];" % (n, base))
        em("%s = sum;" % v)
        em.end()
    em("if (%s && %s == 0) eri_adj_finish(A.adj, qi, aq, g0, g1, g2);" % (active, ls))
    em("return;")
    em.end()


def emit_store_T(em, cp, outs, prec):
    n = cp.n_eriq
    emit_slot(em, "t")
    em("const int64_t obase = oslot * %d;" % n)
    for k, (nm, ix) in enumerate(outs):
        bra, ket = index_parts(cp, *ix)
        em("const int i%d = %s + %s;" % (k, bra, ket))
    if adjoint_form(cp, prec):
        emit_adj_T(em, outs)
    em.block("if (A.out_eri)")
    for k, (nm, ix) in enumerate(outs):
        em("A.out_eri[obase + i%d] = %s;" % (k, nm))
    em.end()
    em("double bmax = 0.0;")
    for nm, _ in outs:
        em("bmax = fmax(bmax, fabs(%s));" % nm)
    em.block("if (A.out_codes)")
    em("const double eps = bmax * A.cn;")
    em("const double inv = eri_inverse_scale(eps);")
    em("if (A.out_scales) A.out_scales[oslot] = eps;")
    em.block("if (A.pack_bits)")
    # packed stream: this lane's codes go to its LDS column, then it packs its quartet's words
    em("const int wide = A.pack_bits > 16;")
    for k, (nm, ix) in enumerate(outs):
        em("eri_stage_code(eri_pack_lds, i%d * (int)blockDim.x + (int)threadIdx.x, wide, "
           "eri_quantize(%s, eps, inv, A.qmax));" % (k, nm))
    em("eri_pack_words(eri_pack_lds, %d, (int)threadIdx.x, (int)blockDim.x, A.pack_bits, A.pack_per, "
       "(int)A.pack_wpq, reinterpret_cast<uint32_t*>(A.out_codes) + oslot * A.pack_wpq * 16);" % n)
    em.end()
    em.block("else")
    for k, (nm, ix) in enumerate(outs):
        em("eri_store_code(A.out_codes, obase + i%d, A.code_bytes, eri_quantize(%s, eps, inv, A.qmax));" % (k, nm))
    em.end()
    em.end()


# ---------------------------------------------------------------------------
# Mode W kernel
# ---------------------------------------------------------------------------
def wave_layout(cp):
    """Lanes per slot, subslot lists of bra indices e.  With one subslot the
    indices are laid out in x-columns (fixed e_y, e_z; e_x = 0, 1, ...), so
    that e - 1_x is always the lane below e: the ket recurrence's coupling
    term along x then moves between lanes by a DPP shift instead of an LDS
    permute."""
    all_e = [e for L in range(cp.Lab + 1) for e in comps(L)]
    if len(all_e) <= 64:
        subs = [[(ex, ey, ez) for ey in range(cp.Lab + 1) for ez in range(cp.Lab + 1 - ey)
                 for ex in range(cp.Lab + 1 - ey - ez)]]
    else:
        subs = [[e for e in all_e if sum(e) % 2 == 0], [e for e in all_e if sum(e) % 2 == 1]]
    ep = max(len(s) for s in subs)
    return subs, ep


def emit_mode_W(cp, prec, name, lds_budget=None, waves=1):
    real = REALS[prec]
    mixed = prec == "mixed"
    em = Emitter()
    a, b, c, d = cp.a, cp.b, cp.c, cp.d
    subs, EP = wave_layout(cp)
    S = len(subs)
    NSLOT = 64 // EP
    if lds_budget is None:
        # 32 KB of HRR staging, or 40 KB where that makes it a single chunk,
        # which the codes pass then reuses (for bras of L >= 3 such kernels are
        # register-bound at four workgroups per CU: the LDS costs no occupancy)
        lds_budget = 40960 if NSLOT <= 3 and lds_chunks(cp, 32768) > 1 and lds_chunks(cp, 40960) == 1 else 32768
    E_T = cp.E_T
    tgt_index = {e: k for k, e in enumerate(E_T)}
    NTE = len(E_T)
    ca, cb, cc, cd = comps(a), comps(b), comps(c), comps(d)
    NCD = len(cc) * len(cd)
    NAB = len(ca) * len(cb)
    CH = min(NCD, max(1, lds_budget // (8 * NSLOT * NTE)))
    NCH = (NCD + CH - 1) // CH
    src_sub = [0] if S == 1 else [1, 0]
    # per-lane table: for each subslot: ex, ey, ez, valid, tgt, src_x, src_y, src_z
    rows = []
    for ls in range(EP):
        row = []
        for s in range(S):
            if ls < len(subs[s]):
                e = subs[s][ls]
                src = []
                for i in range(3):
                    if e[i] >= 1:
                        src.append(subs[src_sub[s]].index(vsub(e, UNIT[i])))
                    else:
                        src.append(ls)
                row += [e[0], e[1], e[2], 1, tgt_index.get(e, -1)] + src
            else:
                row += [0, 0, 0, 0, -1, ls, ls, ls]
        rows.append(row)
    tbl = "eri_tbl_" + name[4:]
    em("// class [%d%d|%d%d] computed as shells %s = [%d%d|%d%d], mode W: %d lanes/slot, %d slot(s), %d subslot(s), %s"
       % (cp.user + (cp.perm, a, b, c, d, EP, NSLOT, S, prec)))
    em("static __constant__ signed char %s[%d][%d] = {" % (tbl, EP, 8 * S))
    for row in rows:
        em("  {" + ", ".join(str(v) for v in row) + "},")
    em("};")
    if waves > 1:
        # at least `waves` wavefronts per SIMD: the register budget halves
        em("__global__ __launch_bounds__(64, %d) void %s(eri_class_args A)" % (waves, name))
    else:
        em("__global__ __launch_bounds__(64) void %s(eri_class_args A)" % name)
    em.block("")
    NF = cp.Ltot + 1 + 17          # staged fields of one primitive quartet
    NSU = max(NSLOT * NTE * CH, NF * 64)
    # one LDS buffer: primitive-quartet staging during the VRR loop, then the
    # HRR staging s_t[slot][target e][cd chunk]
    em("__shared__ double s_u[%d];" % NSU)
    em("double (*s_t)[%d][%d] = reinterpret_cast<double (*)[%d][%d]>(s_u);" % (NTE, CH, NTE, CH))
    G = {"CH": CH, "t": "s_t"}
    nar = narrow_chunking(NSU, NSLOT, NTE, NCD, cp.n_eriq, NCH)
    if nar:
        em("double (*s_tp)[%d][%d] = reinterpret_cast<double (*)[%d][%d]>(s_u);   // packed codes pass"
           % (NTE, nar[0], NTE, nar[0]))
    em("__shared__ double s_red[64];")
    em("const int lane = threadIdx.x;")
    em("const int slot = lane / %d;" % EP)
    em("const int ls = lane - slot * %d;" % EP)
    em("const int64_t qi = (int64_t)blockIdx.x * %d + slot;" % NSLOT)
    em("const bool active = slot < %d && qi < A.n_items;" % NSLOT)
    em("const eri_item it = A.items[active ? qi : 0];")
    em("const bool sb = it.bra < 0, sk = it.ket < 0;   // pair stored in swapped order")
    em("const eri_shell_pair BP = A.pairs[it.bra & 0x7fffffff];")
    em("const eri_shell_pair KP = A.pairs[it.ket & 0x7fffffff];")
    em("const int nbra = active ? BP.nprim : 0;")
    em("const int nket = KP.nprim;")
    em("const int sbase = slot * %d;" % EP)
    # lanes of an unused tail slot read the first slot's staging (never stored)
    em("const int pbase = slot < %d ? sbase : 0;" % NSLOT)
    for s_ in range(S):
        em("const int ex%d = %s[ls][%d], ey%d = %s[ls][%d], ez%d = %s[ls][%d];"
           % (s_, tbl, 8 * s_, s_, tbl, 8 * s_ + 1, s_, tbl, 8 * s_ + 2))
        em("const int tg%d = %s[ls][%d];" % (s_, tbl, 8 * s_ + 4))
        em("const int sx%d = sbase + %s[ls][%d], sy%d = sbase + %s[ls][%d], sz%d = sbase + %s[ls][%d];"
           % (s_, tbl, 8 * s_ + 5, s_, tbl, 8 * s_ + 6, s_, tbl, 8 * s_ + 7))
    # accumulators per subslot
    acc = {}
    for s_ in range(S):
        for f in cp.F_T:
            acc[(s_, f)] = "acc%d_%d%d%d" % ((s_,) + f)
            em("double %s = 0.0;" % acc[(s_, f)])
    # Primitive quartets go through the slot in batches of EP: lane ls does
    # the setup and Boys evaluation of quartet j0 + ls once and stages the
    # results in LDS; then every lane runs the recurrences of each staged
    # quartet.  Trip counts are wave-uniform (max over the slots), staged
    # entries past a slot's own count are zero and contribute nothing.
    em("const int npq = nbra * nket;")
    em("int npq_w = npq;")
    em("for (int o = 32; o > 0; o >>= 1) npq_w = max(npq_w, __shfl_xor(npq_w, o));")
    em.block("for (int j0 = 0; j0 < npq_w; j0 += %d)" % EP)
    em("__syncthreads();")
    em.block("")
    em("double g[%d];" % NF)
    em("#pragma unroll")
    em("for (int q = 0; q < %d; ++q) g[q] = 0.0;" % NF)
    em("const int j = j0 + ls;")
    em.block("if (active && j < npq)")
    em("const int ib = j / nket, ik = j - ib * nket;")
    em("const eri_prim_pair B = A.prims[BP.prim_off + ib];")
    em("const eri_prim_pair K = A.prims[KP.prim_off + ik];")
    em("eri_pq_fp64 S;")
    em("eri_pq_setup(B, K, S);")
    em("double F[%d];" % (cp.Ltot + 1))
    em("eri_boys<%d>(S.T, F);" % cp.Ltot)
    em("#pragma unroll")
    em("for (int m = 0; m <= %d; ++m) g[m] = S.pref * F[m];" % cp.Ltot)
    o = cp.Ltot + 1
    fields = ["B.PA[0]", "B.PA[1]", "B.PA[2]", "S.WP[0]", "S.WP[1]", "S.WP[2]",
              "K.PA[0]", "K.PA[1]", "K.PA[2]", "S.WQ[0]", "S.WQ[1]", "S.WQ[2]",
              "B.hp", "K.hp", "S.hpq", "S.rho_p", "S.rho_q"]
    for k, fld in enumerate(fields):
        em("g[%d] = %s;" % (o + k, fld))
    em.end()
    em("#pragma unroll")
    em("for (int q = 0; q < %d; ++q) s_u[q * 64 + lane] = g[q];" % NF)
    em.end()
    em("__syncthreads();")
    em("const int nb = min(%d, npq_w - j0);" % EP)
    em.block("for (int jj = 0; jj < nb; ++jj)")
    em("const double* u = s_u + pbase + jj;")
    names = ["PAx", "PAy", "PAz", "WPx", "WPy", "WPz", "QCx", "QCy", "QCz", "WQx", "WQy", "WQz",
             "hp", "hq", "hpq", "rp", "rq"]
    for k, nm in enumerate(names):
        em("const %s %s = (%s)u[%d];" % (real, nm, real, 64 * (o + k)))
    MB = cp.Ltot
    for s_ in range(S):
        em("%s c%d[%d], p%d[%d], nx%d[%d];" % (real, s_, MB + 2, s_, MB + 2, s_, MB + 2))
        em("#pragma unroll")
        em("for (int m = 0; m <= %d; ++m) { c%d[m] = (%s)u[64 * m]; p%d[m] = (%s)0; }" % (MB, s_, real, s_, real))
        em("const %s cex%d = (%s)ex%d * hpq, cey%d = (%s)ey%d * hpq, cez%d = (%s)ez%d * hpq;"
           % (real, s_, real, s_, s_, real, s_, s_, real, s_))
    # bra path: step t builds level t along z, then y, then x; lanes already
    # at their |e| apply the identity (pa = 1, wp = 0, c = 0).
    for s in range(S):
        for t in range(1, cp.Lab + 1):
            M = cp.Lcd + cp.Lab - t
            em.block("")
            em("const bool iz = %d <= ez%d;" % (t, s))
            em("const bool iy = !iz && %d <= ez%d + ey%d;" % (t, s, s))
            em("const bool ix = !iz && !iy && %d <= ez%d + ey%d + ex%d;" % (t, s, s, s))
            em("const int nt = iz ? %d : iy ? %d - ez%d : ix ? %d - ez%d - ey%d : 0;" % (t - 1, t - 1, s, t - 1, s, s))
            em("const %s pa = iz ? PAz : iy ? PAy : ix ? PAx : (%s)1;" % (real, real))
            em("const %s wp = iz ? WPz : iy ? WPy : ix ? WPx : (%s)0;" % (real, real))
            em("const %s cc = (%s)nt * hp;" % (real, real))
            em("#pragma unroll")
            em("for (int m = 0; m <= %d; ++m) nx%d[m] = pa * c%d[m] + wp * c%d[m + 1] + cc * (p%d[m] - rp * p%d[m + 1]);"
               % (M, s, s, s, s, s))
            em("#pragma unroll")
            em("for (int m = 0; m <= %d; ++m) { p%d[m] = c%d[m]; c%d[m] = nx%d[m]; }" % (M, s, s, s, s))
            em.end()
    # ket VRR: values V_s(f, m), m <= Lcd - |f|
    V = {}
    # Level order (all f of |f| = k before k + 1): the elements of a level are
    # independent, which gives the scheduler room to hide the permute latency.
    # (A depth-first order along x-chains needs fewer live columns but makes
    # every element wait for the permute of the one before it.)
    kets = [f for L in range(cp.Lcd + 1) for f in comps(L)]
    tset = set(cp.F_T)
    for s in range(S):
        for m in range(cp.Lcd + 1):
            V[(s, ZERO, m)] = "c%d[%d]" % (s, m)
    nvar = 0
    for f in kets:
        if f == ZERO:
            if ZERO in tset:
                for s in range(S):
                    em("%s += %s;" % (acc[(s, f)], ("(double)" + V[(s, f, 0)]) if mixed else V[(s, f, 0)]))
            continue
        L = sum(f)
        i = 0 if f[0] > 0 else (1 if f[1] > 0 else 2)
        ax = "xyz"[i]
        fp = vsub(f, UNIT[i])
        for m in range(cp.Lcd - L + 1):
            for s in range(S):
                nm = "w%d" % nvar
                nvar += 1
                ss = src_sub[s]
                expr = "QC%s * %s + WQ%s * %s" % (ax, V[(s, fp, m)], ax, V[(s, fp, m + 1)])
                if fp[i] >= 1:
                    fpp = vsub(fp, UNIT[i])
                    expr += " + (%s * hq) * (%s - rq * %s)" % (lit(fp[i]), V[(s, fpp, m)], V[(s, fpp, m + 1)])
                if S == 1 and ax == "x":
                    # e - 1_x is the lane below (x-column layout)
                    expr += " + cex0 * eri_lane_below(%s)" % V[(ss, fp, m + 1)]
                else:
                    expr += " + ce%s%d * __shfl(%s, s%s%d)" % (ax, s, V[(ss, fp, m + 1)], ax, s)
                em("const %s %s = %s;" % (real, nm, expr))
                V[(s, f, m)] = nm
        if f in tset:
            for s in range(S):
                v = V[(s, f, 0)]
                em("%s += %s;" % (acc[(s, f)], ("(double)" + v) if mixed else v))
    em.end()
    em.end()
    # HRR
    emit_slot(em, "qi")
    em("const int64_t obase = oslot * %d;" % cp.n_eriq)
    # HRR coefficients: at half the registers (waves > 1) they are formed where
    # they are used (the same products each time, so every pass sees the same
    # bits), since declared once for the epilogue they stayed live and spilled
    # (e.g. [ff|dd] 772 -> 548 bytes per lane, 2.7% faster); at full registers
    # the one declaration spills little ([ff|ff] 164 bytes) and forming them per
    # use measured 3.5% slower
    per_use = waves > 1
    if not per_use:
        emit_hrr_coefs(em, "cd", "KP.AB", cd, real)
        emit_hrr_coefs(em, "ab", "BP.AB", cb, real)
    cd_list = [(ci, di) for ci in cc for di in cd]
    ab_list = [(ai, bi) for ai in ca for bi in cb]

    def ket_hrr_chunk(ch):
        CH, st = G["CH"], G["t"]
        lo, hi = ch * CH, min(NCD, (ch + 1) * CH)
        em("__syncthreads();")
        for s in range(S):
            em.block("if (active && tg%d >= 0)" % s)
            if per_use:
                emit_hrr_coefs(em, "cd", "KP.AB", cd, real)
            for k in range(lo, hi):
                ci, di = cd_list[k]
                expr = hrr_expr(di, ci, lambda f, s=s: "(%s)%s" % (real, acc[(s, f)]), "cd")
                em("%s[slot][tg%d][%d] = (double)(%s);" % (st, s, k - lo, expr))
            em.end()
        em("__syncthreads();")

    stage_base = "slot * %d + " % cp.n_eriq

    def bra_hrr_chunk(ch, pass_no, ctype=None, store_values=True, stage="eri_pack_lds"):
        CH, st = G["CH"], G["t"]
        lo, hi = ch * CH, min(NCD, (ch + 1) * CH)
        n = hi - lo
        if pass_no == 4:
            emit_pack_regs(em, cp, n, EP, "ls", "active && ",
                           lambda e: "(%s)%s[slot][%d][j]" % (real, st, tgt_index[e]), ab_list, stage_base,
                           (lambda: emit_hrr_coefs(em, "ab", "BP.AB", cb, real)) if per_use else None)
            return
        em.block("for (int j = ls; j < %d; j += %d)" % (n, EP))
        em.block("if (active)")
        if per_use:
            emit_hrr_coefs(em, "ab", "BP.AB", cb, real)
        em("const int kcd = %d + j;" % lo)
        for k, (ai, bi) in enumerate(ab_list):
            expr = hrr_expr(bi, ai, lambda e: "(%s)%s[slot][%d][j]" % (real, st, tgt_index[e]), "ab")
            em("const double x%d = (double)(%s);" % (k, expr))
        emit_kx(em, cp)
        if pass_no == 3:
            # codes into the LDS staging: multiply-by-reciprocal quantiser
            # (ctype "fast") or the general one (1/eps overflows somewhere)
            for k in range(len(ab_list)):
                em("const int q%d = %s;" % (k, ("eri_quantize_mul(x%d, inv, A.qmax)" if ctype == "fast" else
                                                "eri_quantize(x%d, eps, inv, A.qmax)") % k))
            emit_stage_codes(em, cp, len(ab_list), stage, stage_base, lambda k: "q%d" % k)
            em.end()
            em.end()
            return
        for k in range(len(ab_list)):
            ia_, ib_ = divmod(k, len(cb))
            bra, _ = index_parts(cp, ia_, ib_, 0, 0)
            ix = "%s + kx" % bra
            if pass_no == 5:
                em("eri_adj_add(A.adj, aq, (int)(%s), x%d, g0, g1, g2);" % (ix, k))
            elif pass_no == 1:
                if store_values is None:
                    em("if (A.out_eri) A.out_eri[obase + %s] = x%d;" % (ix, k))
                elif store_values:
                    em("A.out_eri[obase + %s] = x%d;" % (ix, k))
                em("bmax = fmax(bmax, fabs(x%d));" % k)
            elif ctype is None:
                em("eri_store_code(A.out_codes, obase + %s, A.code_bytes, eri_quantize(x%d, eps, inv, A.qmax));" % (ix, k))
            else:
                em("reinterpret_cast<%s*>(A.out_codes)[obase + %s] = (%s)eri_quantize_mul(x%d, inv, A.qmax);"
                   % (ctype, ix, ctype, k))
        em.end()
        em.end()

    if adjoint_form(cp, prec):
        emit_adj_slot(em, ket_hrr_chunk, bra_hrr_chunk, NCH, "lane", "ls", "sbase", EP, "active", "slot", NSLOT,
                      NSLOT * NTE * CH, NSU - NSLOT * NTE * CH)
    em("double bmax = 0.0;")
    # first pass: b_max, and the FP64 values when requested, decided once (the
    # output pointer is uniform) except in the half-register kernels, where
    # the duplicated code measured slower than a branch per value
    if waves == 1:
        for store in (True, False):
            em.block("if (A.out_eri)" if store else "else")
            for ch in range(NCH):
                ket_hrr_chunk(ch)
                bra_hrr_chunk(ch, 1, store_values=store)
            em.end()
    else:
        for ch in range(NCH):
            ket_hrr_chunk(ch)
            bra_hrr_chunk(ch, 1, store_values=None)
    em("__syncthreads();")
    em("s_red[lane] = bmax;")
    em("__syncthreads();")
    em.block("if (A.out_codes)")
    em("double m = 0.0;")
    em("if (slot < %d) for (int k = 0; k < %d; ++k) m = fmax(m, s_red[sbase + k]);" % (NSLOT, EP))
    em("const double eps = m * A.cn;")
    em("const double inv = eri_inverse_scale(eps);")
    em("if (active && ls == 0 && A.out_scales) A.out_scales[oslot] = eps;")
    # with a single chunk its ket-HRR staging is still in LDS: only the bra
    # HRR is repeated (with several chunks, re-ordering them measured slower)
    # 0: codes over the kernel's own LDS; 1: dynamic LDS; 2: dynamic LDS only
    # for codes wider than 16 bits
    PACK_DYNAMIC_LDS[name] = 0 if NCH == 1 else (2 if nar else 1)
    # a single chunk stages the (int32 at most) codes of every slot over s_u
    assert NCH > 1 or NSU * 8 >= NSLOT * cp.n_eriq * 4, name

    def pack_tail(stage):
        # every lane of the workgroup packs the words of all its quartets
        em("__syncthreads();")
        em("eri_pack_group(%s, %d, (int)min((int64_t)%d, A.n_items - (int64_t)blockIdx.x * %d), A.pack_bits, "
           "A.pack_per, (int)A.pack_wpq, reinterpret_cast<uint32_t*>(A.out_codes), "
           "A.qbase + (int64_t)blockIdx.x * %d, A.ring, lane, 64);"
           % (stage, cp.n_eriq, NSLOT, NSLOT, NSLOT))

    emit_codes_pass(em, NCH, ket_hrr_chunk, bra_hrr_chunk, "__syncthreads_or(__builtin_isinf(inv) ? 1 : 0)", pack_tail,
                    narrow_arg(G, nar, CH))
    em.end()
    em.end()
    return name, em.text()


def xcolumn_waves(cp):
    """The bra indices of an f-f bra (|e| <= 6: 84) split over two
    wavefronts by whole x-columns (fixed e_y, e_z; e_x ascending on
    consecutive lanes), longest columns first, each to the emptier wave."""
    cols = [[(ex, ey, ez) for ex in range(cp.Lab + 1 - ey - ez)]
            for ey in range(cp.Lab + 1) for ez in range(cp.Lab + 1 - ey)]
    cols.sort(key=lambda col: -len(col))
    waves = [[], []]
    for col in cols:
        w = 0 if len(waves[0]) <= len(waves[1]) else 1
        waves[w] += col
    assert max(len(w) for w in waves) <= 64
    return waves


def emit_mode_W2(cp, prec, name, lds_budget=None, waves=1, layout="parity"):
    """Two-subslot classes (|e| <= 6, 84 bra indices) on two wavefronts, one
    bra index per lane, so a lane carries one set of accumulators instead of
    two.  Primitive quartets are staged 64 at a time by the first wave.  One
    LDS pool holds the staging and the exchange during the recurrences, then
    the HRR staging, so two workgroups fit on a CU.

    layout "parity": wave w holds the bra indices of parity w, so the ket
    VRR's coupling term e_i/(2(p+q)) [e-1_i 0|f-1_i 0] always comes from the
    other wave: each ket level's values are exchanged through LDS, with a
    barrier before and after each level's reads.
    layout "xcol": the waves hold whole x-columns (xcolumn_waves), so the
    coupling along x comes from the lane below in the same wave (a DPP
    shift); only the y and z couplings, which lower f along y or z and so
    need values with f_x = 0, go through LDS, into one of two exchange
    buffers used in turn, one barrier per level."""
    real = REALS[prec]
    mixed = prec == "mixed"
    xcol = layout == "xcol"
    em = Emitter()
    a, b, c, d = cp.a, cp.b, cp.c, cp.d
    subs, EP = wave_layout(cp)
    assert len(subs) == 2
    if xcol:
        subs = xcolumn_waves(cp)
    E_T = cp.E_T
    tgt_index = {e: k for k, e in enumerate(E_T)}
    NTE = len(E_T)
    ca, cb, cc, cd = comps(a), comps(b), comps(c), comps(d)
    NCD = len(cc) * len(cd)
    if lds_budget is None:
        # the whole ket-HRR staging in one chunk when it fits 64 KB ([ff|ff]:
        # 59 KB, two workgroups per CU still fit), else 32 KB chunks
        lds_budget = 65536 if NCD * NTE * 8 <= 65536 else 32768
    CH = min(NCD, max(1, lds_budget // (8 * NTE)))
    NCH = (NCD + CH - 1) // CH
    Lcd = cp.Lcd
    # per wave and lane: ex, ey, ez, valid, tgt, src_x, src_y, src_z (src: lane of
    # e - 1_i in the other wave; xcol: flat index 64 w + lane in either wave)
    rows = []
    where = {e: (w, ls) for w in range(2) for ls, e in enumerate(subs[w])}
    for w in range(2):
        other = subs[1 - w]
        for ls in range(64):
            if ls < len(subs[w]):
                e = subs[w][ls]
                if xcol:
                    src = []
                    for i in range(3):
                        if e[i] >= 1:
                            w2, l2 = where[vsub(e, UNIT[i])]
                            if i == 0:
                                assert w2 == w and l2 == ls - 1
                            src.append(64 * w2 + l2)
                        else:
                            src.append(64 * w + ls)
                else:
                    src = [other.index(vsub(e, UNIT[i])) if e[i] >= 1 else ls for i in range(3)]
                rows.append([e[0], e[1], e[2], 1, tgt_index.get(e, -1)] + src)
            else:
                rows.append([0, 0, 0, 0, -1, ls, ls, ls] if not xcol else [0, 0, 0, 0, -1] + [64 * w + ls] * 3)
    tbl = "eri_tbl_" + name[4:]
    em("// class [%d%d|%d%d] computed as shells %s = [%d%d|%d%d], mode W on two waves (%d + %d lanes), %s"
       % (cp.user + (cp.perm, a, b, c, d, len(subs[0]), len(subs[1]), prec)))
    em("static __constant__ signed char %s[128][8] = {" % tbl)   # lane sources 0..127 fit
    for row in rows:
        em("  {" + ", ".join(str(v) for v in row) + "},")
    em("};")
    # exchange slots of one level: values (f, m) with |f| = L - 1, 1 <= m <= Lcd - L + 1
    # (xcol: only f with f_x = 0, the ones the y and z couplings read)
    xidx = {}
    NX = 1
    for L in range(1, Lcd + 1):
        k = 0
        for fp in comps(L - 1):
            if xcol and fp[0] > 0:
                continue
            for m in range(1, Lcd - L + 2):
                xidx[(L, fp, m)] = k
                k += 1
        NX = max(NX, k)
    NF = cp.Ltot + 1 + 17
    NSU = max(NTE * CH, NF * 64 + 2 * NX * 64 * (2 if xcol else 1))
    if waves > 1:
        # `waves` workgroups per CU's SIMD pair: the register budget halves
        em("__global__ __launch_bounds__(128, %d) void %s(eri_class_args A)" % (waves, name))
    else:
        em("__global__ __launch_bounds__(128) void %s(eri_class_args A)" % name)
    em.block("")
    em("__shared__ double s_u[%d];" % NSU)
    if xcol:
        em("double (*s_x)[%d][128] = reinterpret_cast<double (*)[%d][128]>(s_u + %d);   // [buffer][value][64 wave + lane]"
           % (NX, NX, NF * 64))
        em("int xb = 0;   // exchange buffer of the current ket level (uniform)")
    else:
        em("double (*s_x)[%d][64] = reinterpret_cast<double (*)[%d][64]>(s_u + %d);   // [wave][value][lane]"
           % (NX, NX, NF * 64))
    em("__shared__ double s_red[128];")
    em("double (*s_t)[%d] = reinterpret_cast<double (*)[%d]>(s_u);" % (CH, CH))
    G = {"CH": CH, "t": "s_t"}
    nar = narrow_chunking(NSU, 1, NTE, NCD, cp.n_eriq, NCH)
    if nar:
        em("double (*s_tp)[%d] = reinterpret_cast<double (*)[%d]>(s_u);   // packed codes pass" % (nar[0], nar[0]))
    em("const int tid = threadIdx.x;")
    em("const int wv = tid >> 6;")
    em("const int ls = tid & 63;")
    em("const int64_t qi = blockIdx.x;")
    em("const bool active = qi < A.n_items;")
    em("const eri_item it = A.items[active ? qi : 0];")
    em("const bool sb = it.bra < 0, sk = it.ket < 0;   // pair stored in swapped order")
    em("const eri_shell_pair BP = A.pairs[it.bra & 0x7fffffff];")
    em("const eri_shell_pair KP = A.pairs[it.ket & 0x7fffffff];")
    em("const int nbra = active ? BP.nprim : 0;")
    em("const int nket = KP.nprim;")
    em("const int ex0 = %s[tid][0], ey0 = %s[tid][1], ez0 = %s[tid][2];" % (tbl, tbl, tbl))
    em("const int tg0 = %s[tid][4];" % tbl)
    em("const int sx0 = %s[tid][5], sy0 = %s[tid][6], sz0 = %s[tid][7];" % (tbl, tbl, tbl))
    acc = {}
    for f in cp.F_T:
        acc[f] = "acc_%d%d%d" % f
        em("double %s = 0.0;" % acc[f])
    em("const int npq = nbra * nket;   // one quartet per workgroup: uniform")
    em.block("for (int j0 = 0; j0 < npq; j0 += 64)")
    em("__syncthreads();")
    em.block("if (wv == 0)")
    em("double g[%d];" % NF)
    em("#pragma unroll")
    em("for (int q = 0; q < %d; ++q) g[q] = 0.0;" % NF)
    em("const int j = j0 + ls;")
    em.block("if (j < npq)")
    em("const int ib = j / nket, ik = j - ib * nket;")
    em("const eri_prim_pair B = A.prims[BP.prim_off + ib];")
    em("const eri_prim_pair K = A.prims[KP.prim_off + ik];")
    em("eri_pq_fp64 S;")
    em("eri_pq_setup(B, K, S);")
    em("double F[%d];" % (cp.Ltot + 1))
    em("eri_boys<%d>(S.T, F);" % cp.Ltot)
    em("#pragma unroll")
    em("for (int m = 0; m <= %d; ++m) g[m] = S.pref * F[m];" % cp.Ltot)
    o = cp.Ltot + 1
    fields = ["B.PA[0]", "B.PA[1]", "B.PA[2]", "S.WP[0]", "S.WP[1]", "S.WP[2]",
              "K.PA[0]", "K.PA[1]", "K.PA[2]", "S.WQ[0]", "S.WQ[1]", "S.WQ[2]",
              "B.hp", "K.hp", "S.hpq", "S.rho_p", "S.rho_q"]
    for k, fld in enumerate(fields):
        em("g[%d] = %s;" % (o + k, fld))
    em.end()
    em("#pragma unroll")
    em("for (int q = 0; q < %d; ++q) s_u[q * 64 + ls] = g[q];" % NF)
    em.end()
    em("__syncthreads();")
    em("const int nb = min(64, npq - j0);")
    em.block("for (int jj = 0; jj < nb; ++jj)")
    em("const double* u = s_u + jj;")
    names = ["PAx", "PAy", "PAz", "WPx", "WPy", "WPz", "QCx", "QCy", "QCz", "WQx", "WQy", "WQz",
             "hp", "hq", "hpq", "rp", "rq"]
    for k, nm in enumerate(names):
        em("const %s %s = (%s)u[%d];" % (real, nm, real, 64 * (o + k)))
    MB = cp.Ltot
    em("%s c0[%d], p0[%d], nx0[%d];" % (real, MB + 2, MB + 2, MB + 2))
    em("#pragma unroll")
    em("for (int m = 0; m <= %d; ++m) { c0[m] = (%s)u[64 * m]; p0[m] = (%s)0; }" % (MB, real, real))
    em("const %s cex0 = (%s)ex0 * hpq, cey0 = (%s)ey0 * hpq, cez0 = (%s)ez0 * hpq;" % (real, real, real, real))
    for t in range(1, cp.Lab + 1):
        M = cp.Lcd + cp.Lab - t
        em.block("")
        em("const bool iz = %d <= ez0;" % t)
        em("const bool iy = !iz && %d <= ez0 + ey0;" % t)
        em("const bool ix = !iz && !iy && %d <= ez0 + ey0 + ex0;" % t)
        em("const int nt = iz ? %d : iy ? %d - ez0 : ix ? %d - ez0 - ey0 : 0;" % (t - 1, t - 1, t - 1))
        em("const %s pa = iz ? PAz : iy ? PAy : ix ? PAx : (%s)1;" % (real, real))
        em("const %s wp = iz ? WPz : iy ? WPy : ix ? WPx : (%s)0;" % (real, real))
        em("const %s cc = (%s)nt * hp;" % (real, real))
        em("#pragma unroll")
        em("for (int m = 0; m <= %d; ++m) nx0[m] = pa * c0[m] + wp * c0[m + 1] + cc * (p0[m] - rp * p0[m + 1]);" % M)
        em("#pragma unroll")
        em("for (int m = 0; m <= %d; ++m) { p0[m] = c0[m]; c0[m] = nx0[m]; }" % M)
        em.end()
    # ket VRR by levels; the coupling term of level L reads the other wave's
    # level L - 1 values from LDS
    V = {}
    for m in range(Lcd + 1):
        V[(ZERO, m)] = "c0[%d]" % m
    tset = set(cp.F_T)
    if ZERO in tset:
        em("%s += %s;" % (acc[ZERO], ("(double)" + V[(ZERO, 0)]) if mixed else V[(ZERO, 0)]))
    nvar = 0
    for L in range(1, Lcd + 1):
        if xcol:
            # buffers alternate level by level (and across primitive quartets):
            # a wave past this level's barrier has seen the other finish
            # reading the buffer it is about to write
            em("xb ^= 1;")
            for fp in comps(L - 1):
                if fp[0] > 0:
                    continue
                for m in range(1, Lcd - L + 2):
                    em("s_x[xb][%d][tid] = (double)%s;" % (xidx[(L, fp, m)], V[(fp, m)]))
            em("__syncthreads();")
        else:
            em("__syncthreads();   // the other wave has read the previous exchange")
            for fp in comps(L - 1):
                for m in range(1, Lcd - L + 2):
                    em("s_x[wv][%d][ls] = (double)%s;" % (xidx[(L, fp, m)], V[(fp, m)]))
            em("__syncthreads();")
        for f in comps(L):
            i = 0 if f[0] > 0 else (1 if f[1] > 0 else 2)
            ax = "xyz"[i]
            fp = vsub(f, UNIT[i])
            for m in range(Lcd - L + 1):
                nm = "w%d" % nvar
                nvar += 1
                expr = "QC%s * %s + WQ%s * %s" % (ax, V[(fp, m)], ax, V[(fp, m + 1)])
                if fp[i] >= 1:
                    fpp = vsub(fp, UNIT[i])
                    expr += " + (%s * hq) * (%s - rq * %s)" % (lit(fp[i]), V[(fpp, m)], V[(fpp, m + 1)])
                if xcol and i == 0:
                    expr += " + cex0 * eri_lane_below(%s)" % V[(fp, m + 1)]
                elif xcol:
                    expr += " + ce%s0 * (%s)s_x[xb][%d][s%s0]" % (ax, real, xidx[(L, fp, m + 1)], ax)
                else:
                    expr += " + ce%s0 * (%s)s_x[wv ^ 1][%d][s%s0]" % (ax, real, xidx[(L, fp, m + 1)], ax)
                em("const %s %s = %s;" % (real, nm, expr))
                V[(f, m)] = nm
            if f in tset:
                v = V[(f, 0)]
                em("%s += %s;" % (acc[f], ("(double)" + v) if mixed else v))
    em.end()
    em.end()
    # HRR: ket per lane into s_t rows, bra over all 128 threads
    emit_slot(em, "qi")
    em("const int64_t obase = oslot * %d;" % cp.n_eriq)
    # HRR coefficients: at half the registers (waves > 1) they are formed where
    # they are used (the same products each time, so every pass sees the same
    # bits), since declared once for the epilogue they stayed live and spilled
    # (e.g. [ff|dd] 772 -> 548 bytes per lane, 2.7% faster); at full registers
    # the one declaration spills little ([ff|ff] 164 bytes) and forming them per
    # use measured 3.5% slower
    per_use = waves > 1
    if not per_use:
        emit_hrr_coefs(em, "cd", "KP.AB", cd, real)
        emit_hrr_coefs(em, "ab", "BP.AB", cb, real)
    cd_list = [(ci, di) for ci in cc for di in cd]
    ab_list = [(ai, bi) for ai in ca for bi in cb]

    def ket_hrr_chunk(ch):
        CH, st = G["CH"], G["t"]
        lo, hi = ch * CH, min(NCD, (ch + 1) * CH)
        em("__syncthreads();")
        em.block("if (active && tg0 >= 0)")
        if per_use:
            emit_hrr_coefs(em, "cd", "KP.AB", cd, real)
        for k in range(lo, hi):
            ci, di = cd_list[k]
            expr = hrr_expr(di, ci, lambda f: "(%s)%s" % (real, acc[f]), "cd")
            em("%s[tg0][%d] = (double)(%s);" % (st, k - lo, expr))
        em.end()
        em("__syncthreads();")

    stage_base = ""

    def bra_hrr_chunk(ch, pass_no, ctype=None, store_values=True, stage="eri_pack_lds"):
        CH, st = G["CH"], G["t"]
        lo, hi = ch * CH, min(NCD, (ch + 1) * CH)
        n = hi - lo
        if pass_no == 4:
            emit_pack_regs(em, cp, n, 128, "tid", "active && ",
                           lambda e: "(%s)%s[%d][j]" % (real, st, tgt_index[e]), ab_list, stage_base,
                           (lambda: emit_hrr_coefs(em, "ab", "BP.AB", cb, real)) if per_use else None)
            return
        em.block("for (int j = tid; j < %d; j += 128)" % n)
        em.block("if (active)")
        if per_use:
            emit_hrr_coefs(em, "ab", "BP.AB", cb, real)
        em("const int kcd = %d + j;" % lo)
        for k, (ai, bi) in enumerate(ab_list):
            expr = hrr_expr(bi, ai, lambda e: "(%s)%s[%d][j]" % (real, st, tgt_index[e]), "ab")
            em("const double x%d = (double)(%s);" % (k, expr))
        emit_kx(em, cp)
        if pass_no == 3:
            # codes into the LDS staging: multiply-by-reciprocal quantiser
            # (ctype "fast") or the general one (1/eps overflows somewhere)
            for k in range(len(ab_list)):
                em("const int q%d = %s;" % (k, ("eri_quantize_mul(x%d, inv, A.qmax)" if ctype == "fast" else
                                                "eri_quantize(x%d, eps, inv, A.qmax)") % k))
            emit_stage_codes(em, cp, len(ab_list), stage, stage_base, lambda k: "q%d" % k)
            em.end()
            em.end()
            return
        for k in range(len(ab_list)):
            ia_, ib_ = divmod(k, len(cb))
            bra, _ = index_parts(cp, ia_, ib_, 0, 0)
            ix = "%s + kx" % bra
            if pass_no == 5:
                em("eri_adj_add(A.adj, aq, (int)(%s), x%d, g0, g1, g2);" % (ix, k))
            elif pass_no == 1:
                if store_values is None:
                    em("if (A.out_eri) A.out_eri[obase + %s] = x%d;" % (ix, k))
                elif store_values:
                    em("A.out_eri[obase + %s] = x%d;" % (ix, k))
                em("bmax = fmax(bmax, fabs(x%d));" % k)
            elif ctype is None:
                em("eri_store_code(A.out_codes, obase + %s, A.code_bytes, eri_quantize(x%d, eps, inv, A.qmax));" % (ix, k))
            else:
                em("reinterpret_cast<%s*>(A.out_codes)[obase + %s] = (%s)eri_quantize_mul(x%d, inv, A.qmax);"
                   % (ctype, ix, ctype, k))
        em.end()
        em.end()

    if adjoint_form(cp, prec):
        emit_adj_slot(em, ket_hrr_chunk, bra_hrr_chunk, NCH, "tid", "tid", "0", 128, "active", "0", 1,
                      NTE * CH, NSU - NTE * CH)
    em("double bmax = 0.0;")
    # first pass: b_max, and the FP64 values when requested (decided once:
    # the output pointer is uniform)
    for store in (True, False):
        em.block("if (A.out_eri)" if store else "else")
        for ch in range(NCH):
            ket_hrr_chunk(ch)
            bra_hrr_chunk(ch, 1, store_values=store)
        em.end()
    em("__syncthreads();")
    em("s_red[tid] = bmax;")
    em("__syncthreads();")
    em.block("if (A.out_codes)")
    em("double m = 0.0;")
    em("for (int k = 0; k < 128; ++k) m = fmax(m, s_red[k]);")
    em("const double eps = m * A.cn;")
    em("const double inv = eri_inverse_scale(eps);")
    em("if (active && tid == 0 && A.out_scales) A.out_scales[oslot] = eps;")
    # with a single chunk its ket-HRR staging is still in LDS: only the bra
    # HRR is repeated (with several chunks, re-ordering them measured slower)
    PACK_DYNAMIC_LDS[name] = 0 if NCH == 1 else (2 if nar else 1)
    # a single chunk stages the (int32 at most) codes over s_u
    assert NCH > 1 or NSU * 8 >= cp.n_eriq * 4, name

    def pack_tail(stage):
        em("__syncthreads();")
        em("eri_pack_group(%s, %d, active ? 1 : 0, A.pack_bits, A.pack_per, (int)A.pack_wpq, "
           "reinterpret_cast<uint32_t*>(A.out_codes), A.qbase + qi, A.ring, tid, 128);"
           % (stage, cp.n_eriq))

    emit_codes_pass(em, NCH, ket_hrr_chunk, bra_hrr_chunk, "__builtin_isinf(inv) ? 1 : 0", pack_tail,
                    narrow_arg(G, nar, CH))
    em.end()
    em.end()
    return name, em.text()


def emit_class(cp, prec, alt=False, occupancy=1):
    name = kernel_name(prec, cp.user, alt)
    if cp.mode == "T":
        return name, emit_mode_T(cp, prec, name)[1]
    if two_subslot(cp):
        # One wavefront holding two bra indices per lane (84 indices on 64
        # lanes) is not generated.  Such kernels spill 1-3 KB per lane; two of
        # them ([ff|ff] at half the registers with the HRR staging in four
        # chunks, and the full-register [ff|ff] default once its codes pass had
        # grown) returned wrong values on the GPU in some runs and correct ones
        # in others, while the same generated source matched the oracle on the
        # CPU under an emulation of the wavefront.  No indexing, LDS-size or
        # barrier fault was found by reading them; the cause is not known.
        # Such classes run on two wavefronts (emit_mode_W2) instead.
        raise ValueError("%s: a single wavefront with two bra indices per lane is not generated; "
                         "use the two-wavefront form" % name)
    if occupancy > 1:
        name += "_o%d" % occupancy
        return name, emit_mode_W(cp, prec, name, lds_budget=16384, waves=occupancy)[1]
    return name, emit_mode_W(cp, prec, name)[1]


def lds_chunks(cp, lds_budget):
    """Chunks of the ket-HRR staging of a slot-mapped kernel."""
    subs, EP = wave_layout(cp)
    NSLOT = 64 // EP
    NTE = len(cp.E_T)
    NCD = ncart(cp.c) * ncart(cp.d)
    CH = min(NCD, max(1, lds_budget // (8 * NSLOT * NTE)))
    return (NCD + CH - 1) // CH


def swapped_variant(cp):
    """Classes whose two pairs differ much in size also get the other bra/ket
    order (pairs keep their internal order).  With the large pair on the bra
    the slot's lanes each rebuild a long bra path and the bra HRR has few ket
    indices to spread over; with it on the ket the accumulators are many.
    The plan swaps bra and ket of the class's items when this variant runs."""
    if max(cp.user) > 3 or cp.Lab == cp.Lcd or max(cp.Lab, cp.Lcd) < 4:
        return None
    return ClassPlan(*cp.user, perm=cp.perm[2:] + cp.perm[:2])


def two_subslot(cp):
    """Slot-mapped plans whose bra has more indices than a wavefront has lanes
    (an f-f bra, or a g-d bra of the adjoint: 84 indices)."""
    return cp.mode == "W" and len(wave_layout(cp)[0]) == 2


def occupancy_variant(cp):
    """Slot-mapped classes large enough to be register-bound also get a
    kernel limited to half the registers (two wavefronts per SIMD, half the
    LDS staging); single-subslot classes only (see emit_class)."""
    if cp.mode != "W" or cp.Ltot < 6:
        return False
    return not two_subslot(cp)


def alternate_mode(cp):
    """The other work mapping, where it is worth a timed trial: lane per
    quartet for mid-size classes mapped to slots, slots for the larger
    classes mapped to one lane per quartet."""
    if cp.mode == "W" and cp.n_eriq <= 144 and len(cp.elems) <= 320:
        return "T"
    if cp.mode == "T" and cp.Ltot >= 3:
        return "W"
    return None


HEADER = """// Generated by codegen.py -- class-specialised ERI kernels.
#include "eri_device.h"
"""


# kernel tags (last field of eri_kernel_info): which generated kernel a variant launches
TAG_DEFAULT, TAG_ALT, TAG_OCC2, TAG_TWO_WAVES, TAG_SWAP = 0, 1, 2, 3, 4
TAG_TWO_WAVES_OCC2 = 5
TAG_TWO_WAVES_XCOL_OCC2 = 6
# workgroup Rys kernels (RYSW_VARIANTS): 7 larger batches; 8, 9 twice the threads at 4 or 2 waves per
# SIMD; 10, 11, 12 the node loop not unrolled (at 1 and 2 waves per SIMD, and twice the threads at 2)


def two_wave_form(cp):
    """Slot-mapped plans with two bra indices per lane (an f-f bra) also get
    the two-wavefront kernel."""
    return cp.mode == "W" and len(wave_layout(cp)[0]) == 2 and cp.Lcd >= 2


def w2_info(cp, name, tag):
    per_pq, per_q = cp.flops()
    pk = cp.perm[0] | (cp.perm[1] << 2) | (cp.perm[2] << 4) | (cp.perm[3] << 6)
    return "{(const void*)%s, 1, 128, 1, %d, %d, %d, %d, %d}" % (name, cp.n_eriq, per_pq, per_q, pk, tag)


def kernel_info_init(cp, name, block=64, tag=TAG_DEFAULT):
    subs, EP = wave_layout(cp)
    per_pq, per_q = cp.flops()
    pk = cp.perm[0] | (cp.perm[1] << 2) | (cp.perm[2] << 4) | (cp.perm[3] << 6)
    if cp.mode == "T":
        return "{(const void*)%s, 0, %d, %d, %d, %d, %d, %d, %d}" % (name, block, block, cp.n_eriq, per_pq, per_q,
                                                                      pk, tag)
    return "{(const void*)%s, 1, 64, %d, %d, %d, %d, %d, %d}" % (name, 64 // EP, cp.n_eriq, per_pq, per_q, pk, tag)


def variant_infos(cp, name, tag=TAG_DEFAULT):
    """Launch variants of one kernel: mode T at 64, 128 and 256 quartets per
    workgroup, mode W as generated."""
    if cp.mode == "T":
        return [kernel_info_init(cp, name, b, tag) for b in (64, 128, 256)]
    return [kernel_info_init(cp, name, tag=tag)]


def mixed_fp32_classes():
    """Class ids whose recurrences run in FP32 in FP32-mixed plans (the
    measured table mixed_fp32_classes.json beside this file); the other classes
    run their FP64 kernels in such plans.  FP32 Obara-Saika recurrences lose
    digits to cancellation on long bonds with mixed exponents: beyond small
    angular momenta they miss 1e-7 Ha (up to ~1e-3 Ha for [ff|ff]), and on this
    hardware FP32 without packed instructions issues at the FP64 rate, so the
    FP64 kernel costs those classes nothing in arithmetic rate."""
    import json
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "mixed_fp32_classes.json")) as f:
        return set(int(c) for c in json.load(f)["fp32_classes"])


def generate(outdir, precisions=("fp64",), classes=None, group=8, overrides=None, g_classes=True):
    """Write kernel sources (grouped `group` classes per file, each with a host
    registration function filling its entries of the kernel table) and the
    table TU; returns (list of source files, dict of ClassPlan).  `classes`
    is a list of (La, Lb, Lc, Ld); by default the 256 s-f classes in FP64 and,
    for the classes of mixed_fp32_classes(), in FP32-mixed, plus, in FP64
    only, the classes with one g shell.  The FP32-mixed table holds the FP64
    kernels of the other classes."""
    os.makedirs(outdir, exist_ok=True)
    overrides = overrides or {}
    if classes is None:
        classes = [class_of(c) for c in range(256)]
    fp32_ok = mixed_fp32_classes()
    jobs = [(c, prec) for prec in precisions if prec not in ("rys", "rys32") for c in classes
            if prec != "mixed" or class_id(*c) in fp32_ok]
    if g_classes:
        jobs += [(c, "fp64") for c in G_CLASSES]
    plans = {}
    files = []
    regs = []
    for g in range(0, len(jobs), group):
        chunk = jobs[g:g + group]
        parts = [HEADER, '#include "eri_dispatch.h"']
        reg = {}
        for user, prec in chunk:
            cp = plans.get(user)
            if cp is None:
                cp = ClassPlan(*user, **overrides.get(user, {}))
                plans[user] = cp
            c5 = class_id5(*user)
            lines_ = reg.setdefault(prec, [])
            fp32 = ", 1}" if prec == "mixed" else ", 0}"

            def with_flags(info):
                # fp32 flag, then whether the packed path stages in dynamic LDS
                # (mode T kernels and multi-chunk slot kernels do)
                name_ = info[len("{(const void*)"):].split(",")[0]
                return info[:-1] + fp32[:-1] + ", %d}" % PACK_DYNAMIC_LDS.get(name_, 1)
            if two_subslot(cp):
                # an 84-index bra: the default is the two-wavefront x-column kernel
                name = kernel_name(prec, cp.user)
                parts.append(emit_mode_W2(cp, prec, name, layout="xcol")[1])
                lines_.append("    t[%d] = %s;" % (c5, with_flags(w2_info(cp, name, TAG_DEFAULT))))
                infos = [w2_info(cp, name, TAG_DEFAULT)]
            else:
                name, src = emit_class(cp, prec)
                parts.append(src)
                lines_.append("    t[%d] = %s;" % (c5, with_flags(kernel_info_init(cp, name))))
                infos = variant_infos(cp, name)
            am = alternate_mode(cp) if max(user) <= 3 else None
            if am is not None:
                acp = ClassPlan(*user, mode=am, perm=cp.perm)
                aname, asrc = emit_class(acp, prec, alt=True)
                parts.append(asrc)
                infos += variant_infos(acp, aname, TAG_ALT)
            if max(user) <= 3 and occupancy_variant(cp):
                oname, osrc = emit_class(cp, prec, occupancy=2)
                parts.append(osrc)
                infos += variant_infos(cp, oname, TAG_OCC2)
            scp = swapped_variant(cp)
            if scp is not None:
                sname = kernel_name(prec, cp.user) + "_s"
                if scp.mode == "T":
                    parts.append(emit_mode_T(scp, prec, sname)[1])
                    infos += variant_infos(scp, sname, TAG_SWAP)
                elif two_subslot(scp):
                    parts.append(emit_mode_W2(scp, prec, sname, layout="xcol")[1])
                    infos.append(w2_info(scp, sname, TAG_SWAP))
                else:
                    parts.append(emit_mode_W(scp, prec, sname)[1])
                    infos += variant_infos(scp, sname, TAG_SWAP)
            if max(user) <= 3 and two_wave_form(cp):
                wname = kernel_name(prec, cp.user) + "_w2"
                parts.append(emit_mode_W2(cp, prec, wname)[1])
                infos.append(w2_info(cp, wname, TAG_TWO_WAVES))
                if cp.Lcd <= 4:
                    # small ket: the half-register form spills a few hundred bytes per lane
                    # and runs two workgroups per SIMD pair ([ff|fp]: 7.5 -> 5.0 ms); with a
                    # larger ket, or with bra and ket exchanged, it never beat the others
                    parts.append(emit_mode_W2(cp, prec, wname + "o2", waves=2)[1])
                    infos.append(w2_info(cp, wname + "o2", TAG_TWO_WAVES_OCC2))
                if cp.Lcd <= 4:
                    parts.append(emit_mode_W2(cp, prec, wname + "xo2", waves=2, layout="xcol")[1])
                    infos.append(w2_info(cp, wname + "xo2", TAG_TWO_WAVES_XCOL_OCC2))
            assert len(infos) <= MAXVAR, (user, len(infos))
            for k, info in enumerate(infos):
                lines_.append("    v[%d] = %s;" % (c5 * MAXVAR + k, with_flags(info)))
        for prec, lines_ in reg.items():
            fname = "eri_register_%s_g%03d" % (prec, g // group)
            parts.append("void %s(eri_kernel_info* t, eri_kernel_info* v)\n{\n%s\n}\n" % (fname, "\n".join(lines_)))
            regs.append((prec, fname))
        fn = os.path.join(outdir, "eri_k%03d.hip" % (g // group))
        write_if_changed(fn, "\n".join(parts))
        files.append(fn)
    for rprec in [p_ for p_ in ("rys", "rys32") if p_ in precisions]:
        # Rys-quadrature kernels (classes with L_tot <= RYS_LMAX, one lane per
        # quartet): one TU that alone includes the tables of the Rys rule
        real = REALS[rprec]
        parts = [HEADER, '#include "eri_rys.h"', '#include "eri_dispatch.h"']
        lines_ = []
        for user in classes:
            if sum(user) > RYS_LMAX:
                continue
            cp = plans.get(user) or ClassPlan(*user, **overrides.get(user, {}))
            plans[user] = cp
            name = kernel_name(rprec, cp.user)
            _, src, fpq = emit_mode_R(cp, name, real)
            parts.append(src)
            pk = cp.perm[0] | (cp.perm[1] << 2) | (cp.perm[2] << 4) | (cp.perm[3] << 6)
            c5 = class_id5(*user)
            for k, blk in enumerate((64, 128, 256)):
                info = "{(const void*)%s, 0, %d, %d, %d, %d, %d, %d, %d, %d, 1}" % (
                    name, blk, blk, cp.n_eriq, fpq, 3 * cp.n_eriq, pk, TAG_DEFAULT, int(real == "float"))
                if k == 0:
                    lines_.append("    t[%d] = %s;" % (c5, info))
                lines_.append("    v[%d] = %s;" % (c5 * MAXVAR + k, info))
        fname = "eri_register_%s" % rprec
        parts.append("void %s(eri_kernel_info* t, eri_kernel_info* v)\n{\n%s\n}\n" % (fname, "\n".join(lines_)))
        fn = os.path.join(outdir, "eri_%s.hip" % rprec)
        write_if_changed(fn, "\n".join(parts))
        files.append(fn)
        regs.append((rprec, fname))
        # the larger classes: one workgroup per quartet, grouped by L_tot into
        # translation units of at most 24 classes
        big = sorted((u for u in classes if sum(u) > RYS_LMAX), key=lambda u: (sum(u), class_id(*u)))
        for gi in range(0, len(big), 24):
            parts = [HEADER, '#include "eri_rys.h"', '#include "eri_dispatch.h"']
            lines_ = []
            for user in big[gi:gi + 24]:
                cp = plans.get(user) or ClassPlan(*user, **overrides.get(user, {}))
                plans[user] = cp
                pk = cp.perm[0] | (cp.perm[1] << 2) | (cp.perm[2] << 4) | (cp.perm[3] << 6)
                c5 = class_id5(*user)
                k = 0
                vb = 4 if real == "float" else 8
                for suffix, budget, occ, nts, unroll, tag in RYSW_VARIANTS:
                    if budget != RYSW_LDS and rysw_shape(cp, budget, vb) == rysw_shape(cp, RYSW_LDS, vb):
                        continue   # the larger budget changes nothing for this class
                    name = kernel_name(rprec, cp.user) + suffix
                    _, src, fpq = emit_mode_RW(cp, name, budget, occ, real, nts, unroll)
                    parts.append(src)
                    NT = rysw_shape(cp, budget, vb, nts)[0]
                    info = "{(const void*)%s, 1, %d, 1, %d, %d, %d, %d, %d, %d, 0}" % (
                        name, NT, cp.n_eriq, fpq, 3 * cp.n_eriq, pk, tag, int(real == "float"))
                    if k == 0:
                        lines_.append("    t[%d] = %s;" % (c5, info))
                    lines_.append("    v[%d] = %s;" % (c5 * MAXVAR + k, info))
                    k += 1
            fname = "eri_register_%sw_g%02d" % (rprec, gi // 24)
            parts.append("void %s(eri_kernel_info* t, eri_kernel_info* v)\n{\n%s\n}\n" % (fname, "\n".join(lines_)))
            fn = os.path.join(outdir, "eri_%sw_g%02d.hip" % (rprec, gi // 24))
            write_if_changed(fn, "\n".join(parts))
            files.append(fn)
            regs.append((rprec, fname))
    lines = ['#include "eri_dispatch.h"', "#include <mutex>"]
    for prec, fname in regs:
        lines.append("void %s(eri_kernel_info* t, eri_kernel_info* v);" % fname)
    lines.append("static eri_kernel_info g_fp64[ERI_NCLASS5], g_mixed[ERI_NCLASS5], g_rys[ERI_NCLASS5], "
                 "g_rys32[ERI_NCLASS5];")
    lines.append("static eri_kernel_info v_fp64[ERI_NCLASS5 * ERI_MAXVAR], v_mixed[ERI_NCLASS5 * ERI_MAXVAR],")
    lines.append("    v_rys[ERI_NCLASS5 * ERI_MAXVAR], v_rys32[ERI_NCLASS5 * ERI_MAXVAR];")
    lines.append("static std::once_flag g_once;")
    routed = [class_id5(*c) for c in classes if class_id(*c) not in fp32_ok] if "mixed" in precisions else []
    lines.append("// classes whose FP32-mixed entries are their FP64 kernels")
    lines.append("static const int g_mixed_fp64[] = {%s};" % (", ".join(str(c) for c in routed) or "-1"))
    lines.append("static void fill()")
    lines.append("{")
    lines.append("    std::call_once(g_once, [] {")
    for prec, fname in regs:
        lines.append("        %s(g_%s, v_%s);" % (fname, prec, prec))
    lines.append("        for (int c5 : g_mixed_fp64) {")
    lines.append("            if (c5 < 0) continue;")
    lines.append("            g_mixed[c5] = g_fp64[c5];")
    lines.append("            for (int k = 0; k < ERI_MAXVAR; ++k) v_mixed[c5 * ERI_MAXVAR + k] = v_fp64[c5 * ERI_MAXVAR + k];")
    lines.append("        }")
    lines.append("    });")
    lines.append("}")
    lines.append("const eri_kernel_info* eri_kernel_table(int precision)")
    lines.append("{")
    lines.append("    fill();")
    lines.append("    return precision == 3 ? g_rys32 : precision == 2 ? g_rys : precision == 1 ? g_mixed : g_fp64;")
    lines.append("}")
    lines.append("const eri_kernel_info* eri_kernel_variants(int precision)")
    lines.append("{")
    lines.append("    fill();")
    lines.append("    return precision == 3 ? v_rys32 : precision == 2 ? v_rys : precision == 1 ? v_mixed : v_fp64;")
    lines.append("}")
    fn = os.path.join(outdir, "eri_dispatch_table.hip")
    write_if_changed(fn, "\n".join(lines) + "\n")
    files.append(fn)
    return files, plans


def write_if_changed(fn, text):
    if os.path.exists(fn):
        with open(fn) as f:
            if f.read() == text:
                return
    with open(fn, "w") as f:
        f.write(text)
