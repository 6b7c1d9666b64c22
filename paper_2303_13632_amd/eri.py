"""Python binding of liberi_hip.so (include/eri.h): argument marshalling only.

Every step of the ERI computation and compression runs in the library's HIP
kernels; PyTorch supplies device memory and streams.  If the library has not
been built, loading fails with an error (there is no fallback path).
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liberi_hip.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "eri.h")

ERI_OK = 0
ERI_EINVAL = -1
ERI_EUNSUPPORTED = -2
ERI_ENOMEM = -3
ERI_EHIP = -4
ERI_ESTATE = -5
ERI_FP64 = 0
ERI_FP32_MIXED = 1
ERI_RYS = 2
ERI_RYS_FP32 = 3
PRECISIONS = {"fp64": ERI_FP64, "mixed": ERI_FP32_MIXED, "rys": ERI_RYS, "rys32": ERI_RYS_FP32}

_lib = None


class EriError(RuntimeError):
    def __init__(self, status, where):
        lib = load()
        msg = lib.eri_status_string(status).decode()
        if status == ERI_EHIP:
            msg += " (hipError %d)" % lib.eri_last_hip_error()
        super().__init__("%s: %s" % (where, msg))
        self.status = status


ERI_PLAN_ALL_QUARTETS = 1
ERI_PLAN_PACKED = 2


class PlanOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("bits", ctypes.c_int32),
                ("device", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("schwarz_threshold", ctypes.c_double), ("ring_bytes", ctypes.c_int64),
                ("chunk_quartets", ctypes.c_int64), ("scale_block", ctypes.c_int32),
                ("reserved_opt", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_quartets", ctypes.c_int64), ("n_eri", ctypes.c_int64),
                ("n_pairs", ctypes.c_int64), ("n_prim_pairs", ctypes.c_int64),
                ("n_prim_quartets", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("code_bytes", ctypes.c_int32), ("bits", ctypes.c_int32),
                ("batched", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("class_quartets", ctypes.c_int64 * 256), ("class_ring", ctypes.c_int64 * 256),
                ("class_eri_off", ctypes.c_int64 * 257),
                ("class_quartet_off", ctypes.c_int64 * 257), ("class_flops", ctypes.c_double * 256),
                ("class_variant", ctypes.c_int32 * 256), ("class_mode", ctypes.c_int32 * 256),
                ("class_block", ctypes.c_int32 * 256), ("class_per_block", ctypes.c_int32 * 256),
                ("class_n_variants", ctypes.c_int32 * 256), ("class_tag", ctypes.c_int32 * 256),
                ("class_fp32", ctypes.c_int32 * 256), ("scale_block", ctypes.c_int32),
                ("reserved2", ctypes.c_int32), ("class_scale_off", ctypes.c_int64 * 257),
                ("class_word_off", ctypes.c_int64 * 257)]


_vp = ctypes.c_void_p
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def load():
    """Load the HIP library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liberi_hip.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    lib.eri_plan_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int64, _i32p, _i32p, _f64p, _i64p,
                                    _f64p, _f64p, _i32p, ctypes.c_int64, ctypes.POINTER(PlanOpts)]
    lib.eri_plan_info_get.argtypes = [_vp, ctypes.POINTER(PlanInfo)]
    lib.eri_plan_layout.argtypes = [_vp, _i64p, _i64p]
    lib.eri_plan_quartets.argtypes = [_vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, _i32p]
    lib.eri_compute.argtypes = [_vp, _vp, _vp, _vp, _vp]
    lib.eri_compute_class.argtypes = [_vp, ctypes.c_int32, _vp, _vp, _vp, _vp]
    lib.eri_compute_noalloc.argtypes = [_vp, _vp, _vp, _vp, _vp]
    lib.eri_compress.argtypes = [ctypes.c_int32, _vp, ctypes.c_int64, _vp, _vp, _vp, _vp]
    lib.eri_decompress.argtypes = [ctypes.c_int32, _vp, _vp, ctypes.c_int64, _vp, _vp, _vp]
    lib.eri_backward.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int64, _vp, _vp, _vp]
    lib.eri_plan_tune.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_char_p]
    lib.eri_plan_set_variants.argtypes = [_vp, _i32p]
    lib.eri_pack.argtypes = [ctypes.c_int32, _vp, ctypes.c_int64, _vp, _vp, ctypes.c_int64, _vp, _vp]
    lib.eri_unpack.argtypes = [ctypes.c_int32, _vp, ctypes.c_int64, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.eri_plan_set_geometry.argtypes = [_vp, _vp, _vp]
    lib.eri_decompress_host.argtypes = [ctypes.c_int32, _vp, _vp, ctypes.c_int64, _vp, _vp, ctypes.c_int32]
    lib.eri_unpack_host.argtypes = [ctypes.c_int32, _vp, ctypes.c_int64, _vp, _vp, _vp, _vp, _vp, ctypes.c_int32]
    lib.eri_plan_destroy.argtypes = [_vp]
    lib.eri_plan_destroy.restype = None
    lib.eri_status_string.argtypes = [ctypes.c_int]
    lib.eri_status_string.restype = ctypes.c_char_p
    lib.eri_last_hip_error.restype = ctypes.c_int
    _lib = lib
    return lib


def declared_symbols():
    """Function names declared in include/eri.h."""
    import re
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(eri_\w+)\s*\(", txt, re.M)))


def _check(rc, where):
    if rc != ERI_OK:
        raise EriError(rc, where)


def code_dtype(bits):
    import torch
    if bits <= 0:
        return None
    return torch.int8 if bits <= 8 else torch.int16 if bits <= 16 else torch.int32


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A plan over the quartets of a shell set (see include/eri.h).

    quartets=None plans every unique quartet whose Schwarz bound reaches
    `schwarz`; its outputs form per-class rings bounded by `ring_bytes`."""

    def __init__(self, shells, quartets, precision="fp64", bits=16, device=0, schwarz=1e-10,
                 ring_bytes=0, chunk_quartets=0, scale_block=1, packed=False):
        lib = load()
        self.shells = shells
        self.batched = quartets is None
        q = np.zeros((0, 4), dtype=np.int32) if self.batched else \
            np.ascontiguousarray(quartets, dtype=np.int32).reshape(-1, 4)
        self.quartets = q
        self.precision = precision
        self.bits = int(bits)
        self.device = int(device)
        self.packed = bool(packed)
        opts = PlanOpts(PRECISIONS[precision], self.bits, self.device,
                        (ERI_PLAN_ALL_QUARTETS if self.batched else 0) | (ERI_PLAN_PACKED if packed else 0),
                        float(schwarz),
                        int(ring_bytes), int(chunk_quartets), int(scale_block), 0)
        h = _vp()
        L = np.ascontiguousarray(shells["L"], dtype=np.int32)
        K = np.ascontiguousarray(shells["K"], dtype=np.int32)
        xyz = np.ascontiguousarray(shells["xyz"], dtype=np.float64).reshape(-1)
        off = np.ascontiguousarray(shells["off"], dtype=np.int64)
        ex = np.ascontiguousarray(shells["exps"], dtype=np.float64)
        co = np.ascontiguousarray(shells["coefs"], dtype=np.float64)
        if len(ex) == 0:
            ex = np.zeros(1)
            co = np.zeros(1)
        qarg = None if self.batched else (q.reshape(-1) if len(q) else np.zeros(4, dtype=np.int32))
        if qarg is None:
            lib.eri_plan_create.argtypes = lib.eri_plan_create.argtypes[:8] + [_vp] + lib.eri_plan_create.argtypes[9:]
        else:
            lib.eri_plan_create.argtypes = lib.eri_plan_create.argtypes[:8] + [_i32p] + lib.eri_plan_create.argtypes[9:]
        rc = lib.eri_plan_create(ctypes.byref(h), len(L), L, K, xyz, off, ex, co, qarg, len(q), ctypes.byref(opts))
        _check(rc, "eri_plan_create")
        self._h = h
        info = PlanInfo()
        _check(lib.eri_plan_info_get(h, ctypes.byref(info)), "eri_plan_info_get")
        self.n_quartets = info.n_quartets
        self.n_eri = info.n_eri
        self.n_prim_quartets = info.n_prim_quartets
        self.n_pairs = info.n_pairs
        self.n_prim_pairs = info.n_prim_pairs
        self.device_bytes = info.device_bytes
        self.code_bytes = info.code_bytes
        self.class_quartets = np.array(info.class_quartets[:], dtype=np.int64)
        self.class_ring = np.array(info.class_ring[:], dtype=np.int64)
        self.class_eri_off = np.array(info.class_eri_off[:], dtype=np.int64)
        self.class_quartet_off = np.array(info.class_quartet_off[:], dtype=np.int64)
        self.class_scale_off = np.array(info.class_scale_off[:], dtype=np.int64)
        self.scale_block = int(info.scale_block)
        self.class_word_off = np.array(info.class_word_off[:], dtype=np.int64)
        self.class_flops = np.array(info.class_flops[:], dtype=np.float64)
        self._read_variants(info)
        self._pos = None
        self._eri_off = None

    def _read_variants(self, info=None):
        if info is None:
            info = PlanInfo()
            _check(load().eri_plan_info_get(self._h, ctypes.byref(info)), "eri_plan_info_get")
        self.class_variant = np.array(info.class_variant[:], dtype=np.int32)
        self.class_mode = np.array(info.class_mode[:], dtype=np.int32)
        self.class_block = np.array(info.class_block[:], dtype=np.int32)
        self.class_per_block = np.array(info.class_per_block[:], dtype=np.int32)
        self.class_n_variants = np.array(info.class_n_variants[:], dtype=np.int32)
        self.class_tag = np.array(info.class_tag[:], dtype=np.int32)
        self.class_fp32 = np.array(info.class_fp32[:], dtype=np.int32)

    def tune(self, sample_quartets=65536, trials=3, cache=None, stream=None):
        """eri_plan_tune: time each class's launch variants on a sample and keep
        the fastest (choices cached in the JSON file `cache` when given)."""
        path = None if cache is None else os.fsencode(cache)
        _check(load().eri_plan_tune(self._h, _stream(stream), int(sample_quartets), int(trials), path),
               "eri_plan_tune")
        self._read_variants()
        return self.class_variant.copy()

    def set_variants(self, variants):
        v = np.ascontiguousarray(variants, dtype=np.int32)
        if v.shape != (256,):
            raise ValueError("256 variants expected")
        _check(load().eri_plan_set_variants(self._h, v), "eri_plan_set_variants")
        self._read_variants()

    def kernel_name(self, cid):
        """Name of the kernel a class launch uses (variant included)."""
        if self.precision in ("rys", "rys32"):
            return "eri_%s_c%03d%s" % (self.precision, cid, KERNEL_TAG_SUFFIX[int(self.class_tag[cid])])
        prec = "mixed" if self.class_fp32[cid] else "fp64"
        return "eri_%s_c%03d%s" % (prec, cid, KERNEL_TAG_SUFFIX[int(self.class_tag[cid])])

    def layout(self):
        """(pos, eri_off) per user quartet (plan position, first ERI)."""
        if self._pos is None:
            n = int(self.n_quartets)
            pos = np.zeros(max(n, 1), dtype=np.int64)
            eoff = np.zeros(max(n, 1), dtype=np.int64)
            _check(load().eri_plan_layout(self._h, pos, eoff), "eri_plan_layout")
            self._pos, self._eri_off = pos[:n], eoff[:n]
        return self._pos, self._eri_off

    @property
    def out_values(self):
        """Length of the value/code arrays (plan order, rings included)."""
        return int(self.class_eri_off[256])

    @property
    def out_blocks(self):
        """Length of the scale array (one scale per block of scale_block quartets)."""
        return int(self.class_scale_off[256])

    def alloc(self, eri=True, codes=True):
        import torch
        dev = torch.device("cuda", self.device)
        out_eri = torch.empty(max(self.out_values, 1), dtype=torch.float64, device=dev) if eri else None
        out_codes = out_scales = None
        if codes and self.bits > 0 and self.packed:
            # the packed stream: 64-byte words, as int64 lanes
            out_codes = torch.empty(max(8 * int(self.class_word_off[256]), 8), dtype=torch.int64, device=dev)
            out_scales = torch.empty(max(self.out_blocks, 1), dtype=torch.float64, device=dev)
        elif codes and self.bits > 0:
            out_codes = torch.empty(max(self.out_values, 1), dtype=code_dtype(self.bits), device=dev)
            out_scales = torch.empty(max(self.out_blocks, 1), dtype=torch.float64, device=dev)
        return out_eri, out_codes, out_scales

    def class_quartet_list(self, cid, first=0, count=None):
        """Shell quartets of class `cid` in output order (int32 [count, 4])."""
        n = int(self.class_quartets[cid])
        count = n - first if count is None else count
        out = np.zeros(max(4 * count, 4), dtype=np.int32)
        _check(load().eri_plan_quartets(self._h, int(cid), int(first), int(count), out), "eri_plan_quartets")
        return out[: 4 * count].reshape(-1, 4)

    def compute(self, out_eri=None, out_codes=None, out_scales=None, stream=None):
        _check(load().eri_compute(self._h, _stream(stream), _ptr(out_eri), _ptr(out_codes), _ptr(out_scales)),
               "eri_compute")

    def compute_noalloc(self, out_eri=None, out_codes=None, out_scales=None, stream=None):
        """eri_compute_noalloc: the same outputs with no device allocation (static scratch)."""
        _check(load().eri_compute_noalloc(self._h, _stream(stream), _ptr(out_eri), _ptr(out_codes), _ptr(out_scales)),
               "eri_compute_noalloc")

    def compute_class(self, cid, out_eri=None, out_codes=None, out_scales=None, stream=None):
        _check(load().eri_compute_class(self._h, int(cid), _stream(stream), _ptr(out_eri), _ptr(out_codes),
                                        _ptr(out_scales)), "eri_compute_class")

    @property
    def n_prims(self):
        """Length of the exponent array (gradients per primitive)."""
        return len(self.shells["exps"])

    @property
    def nbf(self):
        """Cartesian basis functions of the shell set."""
        return int(sum(_ncart(l) for l in self.shells["L"]))

    def backward(self, dl=None, density=None, grad_centers=None, grad_exps=None, energy=None, stream=None,
                 energy_only=False):
        """eri_backward: adds dL/dxyz and dL/dexps of L = sum w Gbar (ab|cd)
        (Gbar = dl in the plan layout, or D D from a density) into the given
        device tensors, allocating zeroed ones when None.  Returns
        (grad_centers [n_shells, 3], grad_exps [n_prims], energy [1])."""
        import torch
        dev = torch.device("cuda", self.device)
        if grad_centers is None and not energy_only:
            grad_centers = torch.zeros((len(self.shells["L"]), 3), dtype=torch.float64, device=dev)
        if grad_exps is None and not energy_only:
            grad_exps = torch.zeros(max(self.n_prims, 1), dtype=torch.float64, device=dev)
        if energy is None:
            energy = torch.zeros(1, dtype=torch.float64, device=dev)
        for t in (dl, density, grad_centers, grad_exps, energy):
            if t is not None and (t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda):
                raise ValueError("eri_backward takes contiguous float64 device tensors")
        if dl is not None and dl.numel() < self.out_values:
            raise ValueError("dl holds %d values, the plan layout %d" % (dl.numel(), self.out_values))
        nbf = 0 if density is None else int(density.shape[0])
        _check(load().eri_backward(self._h, _stream(stream), _ptr(dl), _ptr(density), nbf, _ptr(grad_centers),
                                   _ptr(grad_exps), _ptr(energy)), "eri_backward")
        return grad_centers, None if grad_exps is None else grad_exps[: self.n_prims], energy

    def check_parameters(self, centers, exps):
        """The plan's integrals are those of its shell set: autograd inputs
        must hold the same centres and exponents."""
        c = centers.detach().to("cpu", torch_float64()).numpy().reshape(-1, 3)
        e = exps.detach().to("cpu", torch_float64()).numpy().reshape(-1)
        if not (np.array_equal(c, np.asarray(self.shells["xyz"], dtype=np.float64).reshape(-1, 3)) and
                np.array_equal(e, np.asarray(self.shells["exps"], dtype=np.float64))):
            raise ValueError("centres/exponents differ from the plan's shell set; build a new plan")

    def to_user(self, values):
        """Plan-order per-ERI array (numpy) -> user order (concatenated blocks)."""
        pos, eoff = self.layout()
        L = self.shells["L"]
        sizes = np.array([_ncart(L[a]) * _ncart(L[b]) * _ncart(L[c]) * _ncart(L[d]) for a, b, c, d in self.quartets],
                         dtype=np.int64)
        idx = np.concatenate([np.arange(o, o + s) for o, s in zip(eoff, sizes)]) if len(sizes) else np.zeros(0, np.int64)
        return values[idx]

    def scales_to_user(self, scales):
        pos, _ = self.layout()
        return scales[pos]

    def set_geometry(self, xyz=None, exps=None):
        """eri_plan_set_geometry: new centres [n_shells, 3] and/or exponents for
        the same quartet set (screening and orientation kept)."""
        x = None if xyz is None else np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1)
        e = None if exps is None else np.ascontiguousarray(exps, dtype=np.float64).reshape(-1)
        if x is not None and len(x) != 3 * len(self.shells["L"]):
            raise ValueError("xyz needs 3 values per shell")
        if e is not None and len(e) != len(self.shells["exps"]):
            raise ValueError("exps needs one value per primitive")
        _check(load().eri_plan_set_geometry(self._h, None if x is None else x.ctypes.data_as(ctypes.c_void_p),
                                            None if e is None else e.ctypes.data_as(ctypes.c_void_p)),
               "eri_plan_set_geometry")
        sh = dict(self.shells)
        if x is not None:
            sh["xyz"] = x.reshape(-1, 3).copy()
        if e is not None:
            sh["exps"] = e.copy()
        self.shells = sh

    def close(self):
        if getattr(self, "_h", None):
            load().eri_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# Name suffix of the generated kernel of each variant tag (eri_plan_info.class_tag)
KERNEL_TAG_SUFFIX = {0: "", 1: "_a", 2: "_o2", 3: "_w2", 4: "_s", 5: "_w2o2", 6: "_w2xo2", 7: "_b", 8: "_w", 9: "_wo2",
                     10: "_n", 11: "_no2", 12: "_nwo2"}


def _ncart(L):
    return (int(L) + 1) * (int(L) + 2) // 2


def compress(bits, eri, block_off, codes=None, scales=None, stream=None):
    """eqs. 9-10 on device tensors: returns (codes, scales)."""
    import torch
    nb = block_off.numel() - 1
    if codes is None:
        codes = torch.empty(eri.numel(), dtype=code_dtype(bits), device=eri.device)
    if scales is None:
        scales = torch.empty(max(nb, 1), dtype=torch.float64, device=eri.device)
    _check(load().eri_compress(int(bits), _ptr(eri), nb, _ptr(block_off), _ptr(codes), _ptr(scales),
                               _stream(stream)), "eri_compress")
    return codes, scales


def decompress(bits, codes, scales, block_off, out=None, stream=None):
    """eq. 11 on device tensors."""
    import torch
    nb = block_off.numel() - 1
    if out is None:
        out = torch.empty(codes.numel(), dtype=torch.float64, device=codes.device)
    _check(load().eri_decompress(int(bits), _ptr(codes), _ptr(scales), nb, _ptr(block_off), _ptr(out),
                                 _stream(stream)), "eri_decompress")
    return out


def torch_float64():
    import torch
    return torch.float64


def _make_autograd():
    import torch

    class ERIFunction(torch.autograd.Function):
        """values = ERIFunction.apply(centers, exps, plan): the plan's FP64 ERIs
        (plan layout) as a differentiable function of the shell centres
        [n_shells, 3] and primitive exponents; backward calls eri_backward."""

        @staticmethod
        def forward(ctx, centers, exps, plan):
            plan.check_parameters(centers, exps)
            out, _, _ = plan.alloc(eri=True, codes=False)
            plan.compute(out)
            ctx.plan = plan
            return out

        @staticmethod
        def backward(ctx, g):
            plan = ctx.plan
            gc, ge, _ = plan.backward(dl=g.to(torch.float64).contiguous())
            return gc, ge, None

    class CoulombEnergy(torch.autograd.Function):
        """E = CoulombEnergy.apply(centers, exps, plan, density): the density
        contraction sum D D (ab|cd) over the plan's quartets (weighted by their
        degeneracy for all-quartet plans), computed together with its
        gradient in one eri_backward call."""

        @staticmethod
        def forward(ctx, centers, exps, plan, density):
            plan.check_parameters(centers, exps)
            gc, ge, en = plan.backward(density=density.to(torch.float64).contiguous())
            ctx.save_for_backward(gc, ge)
            return en[0].clone()

        @staticmethod
        def backward(ctx, g):
            gc, ge = ctx.saved_tensors
            return g * gc, g * ge, None, None

    return ERIFunction, CoulombEnergy


_autograd = None


def __getattr__(name):
    global _autograd
    if name in ("ERIFunction", "CoulombEnergy"):
        if _autograd is None:
            _autograd = _make_autograd()
        return _autograd[0] if name == "ERIFunction" else _autograd[1]
    raise AttributeError(name)


def packed_word_offsets(bits, block_off):
    """First 512-bit word of every block (n_blocks + 1 entries, host numpy):
    ceil(size / floor(512 / bits)) words per block."""
    per = 512 // int(bits)
    sizes = np.diff(np.asarray(block_off, dtype=np.int64))
    w = np.zeros(len(sizes) + 1, dtype=np.int64)
    w[1:] = np.cumsum((sizes + per - 1) // per)
    return w


def pack(bits, codes, block_off, word_off, packed=None, stream=None):
    """eri_pack on device tensors (block_off, word_off: device int64)."""
    import torch
    nb = block_off.numel() - 1
    n_words = int(word_off[-1].item()) if word_off.numel() else 0
    if packed is None:
        packed = torch.zeros(max(8 * n_words, 8), dtype=torch.int64, device=codes.device)
    _check(load().eri_pack(int(bits), _ptr(codes), nb, _ptr(block_off), _ptr(word_off), n_words, _ptr(packed),
                           _stream(stream)), "eri_pack")
    return packed


def unpack(bits, packed, block_off, word_off, scales=None, codes=True, values=False, stream=None):
    """eri_unpack: returns (int32 codes or None, decompressed values or None)."""
    import torch
    nb = block_off.numel() - 1
    n = int(block_off[-1].item()) if block_off.numel() else 0
    c = torch.empty(max(n, 1), dtype=torch.int32, device=packed.device) if codes else None
    v = torch.empty(max(n, 1), dtype=torch.float64, device=packed.device) if values else None
    _check(load().eri_unpack(int(bits), _ptr(packed), nb, _ptr(block_off), _ptr(word_off), _ptr(scales), _ptr(c),
                             _ptr(v), _stream(stream)), "eri_unpack")
    return c, v


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def decompress_host(bits, codes, scales, block_off, out=None, n_threads=0):
    """eri_decompress_host on host numpy arrays: FP64 values code * eps."""
    codes = np.ascontiguousarray(codes)
    scales = np.ascontiguousarray(scales, dtype=np.float64)
    block_off = np.ascontiguousarray(block_off, dtype=np.int64)
    if out is None:
        out = np.empty(len(codes), dtype=np.float64)
    _check(load().eri_decompress_host(int(bits), _np_ptr(codes), _np_ptr(scales), len(block_off) - 1,
                                      _np_ptr(block_off), _np_ptr(out), int(n_threads)), "eri_decompress_host")
    return out


def unpack_host(bits, packed, block_off, word_off, scales=None, codes=True, values=False, n_threads=0):
    """eri_unpack_host on host numpy arrays: (int32 codes or None, values or None)."""
    packed = np.ascontiguousarray(packed)
    block_off = np.ascontiguousarray(block_off, dtype=np.int64)
    word_off = np.ascontiguousarray(word_off, dtype=np.int64)
    n = int(block_off[-1]) if len(block_off) else 0
    c = np.empty(n, dtype=np.int32) if codes else None
    v = np.empty(n, dtype=np.float64) if values else None
    sc = None if scales is None else np.ascontiguousarray(scales, dtype=np.float64)
    _check(load().eri_unpack_host(int(bits), _np_ptr(packed), len(block_off) - 1, _np_ptr(block_off),
                                  _np_ptr(word_off), _np_ptr(sc), _np_ptr(c), _np_ptr(v), int(n_threads)),
           "eri_unpack_host")
    return c, v
