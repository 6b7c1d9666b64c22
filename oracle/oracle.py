"""ctypes binding of the C oracle (eri_oracle.c).

TEST INFRASTRUCTURE: used by the tests, the smoke check and the benchmark's CPU
baseline only.

Conventions (the same as the paper's section II, with the readings noted in
eri_oracle.c):
  * a shell set is given as arrays L[n], K[n], xyz[n,3], off[n+1] (prefix
    offsets into exps/coefs);
  * a quartet is four shell indices (a, b, c, d);
  * quartet t writes its n_ERIQ values row-major over (a, b, c, d) Cartesian
    components, each shell's components ordered x^L first
    (lx = L..0, ly = L-lx..0).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "eri_oracle.c")
_LIB = os.path.join(_HERE, "liberi_oracle.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def build(force=True):
    """Compile the oracle with gcc (-O3, OpenMP, no FMA contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-std=gnu11", "-o", tmp, _SRC, "-lquadmath", "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.oracle_boys.argtypes = [ctypes.c_int, ctypes.c_double, _f64p]
    lib.oracle_rys_rule.argtypes = [ctypes.c_int, ctypes.c_double, _f64p, _f64p]
    lib.oracle_norm.argtypes = [ctypes.c_double, ctypes.c_int]
    lib.oracle_norm.restype = ctypes.c_double
    for name in ("oracle_eri_d", "oracle_eri_q"):
        getattr(lib, name).argtypes = [ctypes.c_int64, _i32p, _i32p, _f64p, _i64p, _f64p, _f64p,
                                       ctypes.c_int64, _i32p, _i64p, _f64p, ctypes.c_int]
    lib.oracle_primitive_block.argtypes = [_i32p, _f64p, _f64p, _f64p]
    lib.oracle_compress.argtypes = [ctypes.c_int, ctypes.c_int64, _i64p, _f64p, _i32p, _f64p]
    lib.oracle_decompress.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _f64p]
    _vp = ctypes.c_void_p
    lib.oracle_gradient.argtypes = [ctypes.c_int64, _i32p, _i32p, _f64p, _i64p, _f64p, _f64p,
                                    ctypes.c_int64, _i32p, _f64p, _vp, _vp, _vp, ctypes.c_int64,
                                    _f64p, _f64p, _f64p, ctypes.c_int]
    _lib = lib
    return lib


def ncart(L):
    return (L + 1) * (L + 2) // 2


def components(L):
    """Cartesian components of a shell, x^L first."""
    return [(lx, ly, L - lx - ly) for lx in range(L, -1, -1) for ly in range(L - lx, -1, -1)]


def boys(mmax, T):
    """F_0..F_mmax at T, evaluated in __float128 and rounded to double."""
    F = np.zeros(mmax + 1)
    if load().oracle_boys(int(mmax), float(T), F) != 0:
        raise ValueError("oracle_boys: bad arguments")
    return F


def rys_rule(n, T):
    """n-point Rys rule (eq. 5): nodes u = t^2 and weights w."""
    u = np.zeros(n)
    w = np.zeros(n)
    if load().oracle_rys_rule(int(n), float(T), u, w) != 0:
        raise ValueError("oracle_rys_rule: bad arguments")
    order = np.argsort(u)
    return u[order], w[order]


def norm(alpha, L):
    """Normalisation N(alpha, L) of eq. 1 (axis-aligned component normalised)."""
    return load().oracle_norm(float(alpha), int(L))


def _eri(fn, shells, quartets, n_threads):
    L = np.ascontiguousarray(shells["L"], dtype=np.int32)
    K = np.ascontiguousarray(shells["K"], dtype=np.int32)
    xyz = np.ascontiguousarray(shells["xyz"], dtype=np.float64).reshape(-1)
    off = np.ascontiguousarray(shells["off"], dtype=np.int64)
    exps = np.ascontiguousarray(shells["exps"], dtype=np.float64)
    coefs = np.ascontiguousarray(shells["coefs"], dtype=np.float64)
    q = np.ascontiguousarray(quartets, dtype=np.int32).reshape(-1, 4)
    nq = q.shape[0]
    sizes = np.array([ncart(L[a]) * ncart(L[b]) * ncart(L[c]) * ncart(L[d]) for a, b, c, d in q],
                     dtype=np.int64)
    out_off = np.zeros(nq, dtype=np.int64)
    if nq:
        out_off[1:] = np.cumsum(sizes)[:-1]
    out = np.zeros(int(sizes.sum()))
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    rc = fn(len(L), L, K, xyz, off, exps, coefs, nq, q.reshape(-1), out_off, out, int(n_threads))
    if rc != 0:
        raise ValueError("oracle_eri: bad arguments (rc=%d)" % rc)
    return out, out_off, sizes


def eri(shells, quartets, n_threads=None):
    """Contracted ERIs of each quartet (double instantiation).

    Returns (values, offsets, sizes): quartet t occupies
    values[offsets[t] : offsets[t] + sizes[t]], row-major (a, b, c, d)."""
    return _eri(load().oracle_eri_d, shells, quartets, n_threads)


def eri_quad(shells, quartets, n_threads=None):
    """Same as eri() but every step in __float128 (referee), rounded at the end."""
    return _eri(load().oracle_eri_q, shells, quartets, n_threads)


def primitive_block(L, R, ex):
    """Unnormalised primitive block for angular momenta L[4], centres R[4,3],
    exponents ex[4] (no normalisation, no coefficients)."""
    L = np.ascontiguousarray(L, dtype=np.int32)
    n = int(np.prod([ncart(int(x)) for x in L]))
    out = np.zeros(n)
    rc = load().oracle_primitive_block(L, np.ascontiguousarray(R, dtype=np.float64).reshape(-1),
                                       np.ascontiguousarray(ex, dtype=np.float64), out)
    if rc != 0:
        raise ValueError("oracle_primitive_block: bad arguments")
    return out


def compress(bits, x, block_off):
    """Eqs. 9-10 per block: returns (codes int32, eps per block)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    block_off = np.ascontiguousarray(block_off, dtype=np.int64)
    nb = len(block_off) - 1
    codes = np.zeros(len(x), dtype=np.int32)
    eps = np.zeros(nb)
    if load().oracle_compress(int(bits), nb, block_off, x, codes, eps) != 0:
        raise ValueError("oracle_compress: bad arguments")
    return codes, eps


def decompress(codes, eps, block_off):
    """Eq. 11: x~ = q * eps."""
    codes = np.ascontiguousarray(codes, dtype=np.int32)
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    block_off = np.ascontiguousarray(block_off, dtype=np.int64)
    out = np.zeros(len(codes))
    if load().oracle_decompress(len(block_off) - 1, block_off, codes, eps, out) != 0:
        raise ValueError("oracle_decompress: bad arguments")
    return out


def gradient(shells, quartets, weights=None, dl=None, density=None, n_threads=None):
    """Analytic gradient of  L = sum_t w_t sum_(abcd) Gbar_t(abcd) (ab|cd)_t
    with Gbar = dl (values in the layout of eri(), i.e. quartet t at its
    offset) or Gbar = D[mu nu] D[lam sig] from a symmetric density over the
    basis functions numbered shell by shell.  Returns (L, dL/dxyz [n, 3],
    dL/dexps [len(exps)]).  All four centres are differentiated explicitly."""
    L = np.ascontiguousarray(shells["L"], dtype=np.int32)
    K = np.ascontiguousarray(shells["K"], dtype=np.int32)
    xyz = np.ascontiguousarray(shells["xyz"], dtype=np.float64).reshape(-1)
    off = np.ascontiguousarray(shells["off"], dtype=np.int64)
    exps = np.ascontiguousarray(shells["exps"], dtype=np.float64)
    coefs = np.ascontiguousarray(shells["coefs"], dtype=np.float64)
    q = np.ascontiguousarray(quartets, dtype=np.int32).reshape(-1, 4)
    nq = q.shape[0]
    w = np.ones(nq) if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    if (dl is None) == (density is None):
        raise ValueError("give exactly one of dl and density")
    keep = []
    dl_off = None
    nbf = 0
    if dl is not None:
        sizes = np.array([ncart(L[a]) * ncart(L[b]) * ncart(L[c]) * ncart(L[d]) for a, b, c, d in q],
                         dtype=np.int64)
        dl_off = np.zeros(max(nq, 1), dtype=np.int64)
        if nq:
            dl_off[1:nq] = np.cumsum(sizes)[:-1]
        dl = np.ascontiguousarray(dl, dtype=np.float64)
        keep += [dl, dl_off]
        dl_p, off_p, d_p = dl.ctypes.data, dl_off.ctypes.data, None
    else:
        density = np.ascontiguousarray(density, dtype=np.float64)
        nbf = density.shape[0]
        keep.append(density)
        dl_p, off_p, d_p = None, None, density.ctypes.data
    gx = np.zeros(3 * len(L))
    ge = np.zeros(max(len(exps), 1))
    en = np.zeros(1)
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    rc = load().oracle_gradient(len(L), L, K, xyz, off, exps, coefs, nq,
                                q.reshape(-1) if nq else np.zeros(4, np.int32), w if nq else np.zeros(1),
                                dl_p, off_p, d_p, nbf, gx, ge, en, int(n_threads))
    if rc != 0:
        raise ValueError("oracle_gradient: bad arguments (rc=%d)" % rc)
    return float(en[0]), gx.reshape(-1, 3), ge[:len(exps)]


def pack(bits, codes, block_off):
    """Packed stream of n-bit codes: 512-bit words of floor(512/n) codes,
    every block (quartet) starting on a new word; code k of a block sits in
    word k // per at bit (k % per) * n of the word (bit 0 = least significant
    bit of the word's first byte), as its n low two's-complement bits.
    Returns (uint8 array of 64-byte words, word offset of each block)."""
    bits = int(bits)
    per = 512 // bits
    codes = np.asarray(codes, dtype=np.int64)
    block_off = np.asarray(block_off, dtype=np.int64)
    sizes = np.diff(block_off)
    word_off = np.zeros(len(sizes) + 1, dtype=np.int64)
    word_off[1:] = np.cumsum((sizes + per - 1) // per)
    out = np.zeros(int(word_off[-1]) * 64, dtype=np.uint8)
    mask = (1 << bits) - 1
    for b in range(len(sizes)):
        for k in range(int(sizes[b])):
            v = int(codes[block_off[b] + k]) & mask
            w = int(word_off[b]) + k // per
            pos = (k % per) * bits
            for t in range(bits):
                if (v >> t) & 1:
                    bit = pos + t
                    out[64 * w + bit // 8] |= np.uint8(1 << (bit % 8))
    return out, word_off


def unpack(bits, packed, block_off):
    """Inverse of pack(): int64 codes, sign-extended from n bits."""
    bits = int(bits)
    per = 512 // bits
    block_off = np.asarray(block_off, dtype=np.int64)
    sizes = np.diff(block_off)
    word_off = np.zeros(len(sizes) + 1, dtype=np.int64)
    word_off[1:] = np.cumsum((sizes + per - 1) // per)
    packed = np.asarray(packed, dtype=np.uint8)
    out = np.zeros(int(block_off[-1]) if len(block_off) else 0, dtype=np.int64)
    for b in range(len(sizes)):
        for k in range(int(sizes[b])):
            w = int(word_off[b]) + k // per
            pos = (k % per) * bits
            v = 0
            for t in range(bits):
                bit = pos + t
                if (int(packed[64 * w + bit // 8]) >> (bit % 8)) & 1:
                    v |= 1 << t
            if v >> (bits - 1):
                v -= 1 << bits
            out[block_off[b] + k] = v
    return out
