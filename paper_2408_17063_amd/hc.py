"""Python binding of libhc (include/hc.h, include/hc_kernels.h).

Argument marshalling only: every operation runs in the library's HIP kernels
(or, for decryption and decompression, its host C++). Device buffers are torch
tensors (int64, reinterpreted as uint64 residues) on the GPU; streams are
torch's current stream. There is no fallback: if libhc.so cannot be loaded,
importing this module raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libhc.so is not built (run paper_2408_17063_amd.build.build())")
# torch first: libhc.so links the HIP runtime torch ships, which must be the one
# loaded (and initialised) in this process
import torch  # noqa: E402,F401
_lib = ctypes.CDLL(LIB_PATH)

c_u8p = ctypes.POINTER(ctypes.c_uint8)
c_u32p = ctypes.POINTER(ctypes.c_uint32)
c_u64p = ctypes.POINTER(ctypes.c_uint64)
c_i64p = ctypes.POINTER(ctypes.c_int64)
c_vp = ctypes.c_void_p

HC_OK, HC_EINVAL, HC_ENOMEM, HC_EDEVICE, HC_ENOKEY, HC_EDECODE, HC_ENOISE, HC_ESCRATCH = 0, -1, -2, -3, -4, -5, -6, -7
DIAG_LAYOUT_AUTO, DIAG_LAYOUT_SPLIT = 0, 1
NOALLOC_SCRATCH_BYTES = 64 << 20


class HcError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        msg = _lib.hc_status_str(status).decode()
        super().__init__("%s: %s (%d)" % (what, msg, status))


class Params(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("p", ctypes.c_uint64), ("L", ctypes.c_uint32),
                ("q_bits", ctypes.c_uint32), ("K", ctypes.c_uint32), ("p_bits", ctypes.c_uint32)]


class CompressInfo(ctypes.Structure):
    _fields_ = [("s", ctypes.c_uint32), ("groups", ctypes.c_uint32), ("streams", ctypes.c_uint32),
                ("bands", ctypes.c_uint32), ("n_ct", ctypes.c_uint32),
                ("n_keyswitch", ctypes.c_uint32), ("n_ptct", ctypes.c_uint64),
                ("n_diag", ctypes.c_uint64), ("level", ctypes.c_uint32),
                ("n_diag_resident", ctypes.c_uint64), ("comp_level", ctypes.c_uint32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


TUNE_MAC_VARIANTS, TUNE_NTT_VARIANTS = 3, 4


class TuneReport(ctypes.Structure):
    _fields_ = [("mac_variant", ctypes.c_uint32), ("ntt_variant", ctypes.c_uint32),
                ("mac_ms", ctypes.c_double * TUNE_MAC_VARIANTS), ("ntt_ms", ctypes.c_double * TUNE_NTT_VARIANTS)]

    def as_dict(self):
        return {"mac_variant": self.mac_variant, "ntt_variant": self.ntt_variant,
                "mac_ms": [round(x, 4) for x in self.mac_ms], "ntt_ms": [round(x, 4) for x in self.ntt_ms]}


class Query(ctypes.Structure):
    _fields_ = [("ct_v", c_vp), ("N", ctypes.c_uint64), ("t_bound", ctypes.c_uint32),
                ("comp_level", ctypes.c_uint32), ("out_level", ctypes.c_uint32), ("ct_out", c_vp),
                ("info", ctypes.POINTER(CompressInfo)), ("status", ctypes.c_int)]


class ServerResult(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int), ("submit_ns", ctypes.c_int64),
                ("start_ns", ctypes.c_int64), ("done_ns", ctypes.c_int64), ("batch_size", ctypes.c_uint32),
                ("info", CompressInfo)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("max_batch_seen", ctypes.c_uint32), ("max_lanes_busy", ctypes.c_uint32)]


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_st = ctypes.c_int
_sig("hc_status_str", ctypes.c_char_p, _st)
_sig("hc_context_create", _st, ctypes.POINTER(Params), ctypes.c_int, ctypes.POINTER(c_vp))
_sig("hc_context_destroy", None, c_vp)
_sig("hc_context_primes", _st, c_vp, c_u64p)
_sig("hc_context_trim", None, c_vp)
_sig("hc_keygen", _st, c_vp, c_u8p, ctypes.POINTER(c_vp), ctypes.POINTER(c_vp))
_sig("hc_sk_destroy", None, c_vp)
_sig("hc_pk_destroy", None, c_vp)
_sig("hc_galois_keygen", _st, c_vp, c_vp, c_u32p, ctypes.c_uint32, c_u8p, ctypes.POINTER(c_vp))
_sig("hc_gk_destroy", None, c_vp)
_sig("hc_plan", _st, c_vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
     c_u32p, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(CompressInfo))
_sig("hc_db_upload", _st, c_vp, c_u32p, ctypes.c_uint32, ctypes.c_uint64, ctypes.POINTER(c_vp))
_sig("hc_db_destroy", None, c_vp)
_sig("hc_encrypt", _st, c_vp, c_vp, c_u32p, c_u8p, c_vp, c_vp)
_sig("hc_compress", _st, c_vp, c_vp, c_vp, c_vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
     c_vp, ctypes.POINTER(CompressInfo), c_vp)
_sig("hc_compress_plain_db", _st, c_vp, c_vp, c_vp, c_vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
     ctypes.c_uint32, c_vp, ctypes.POINTER(CompressInfo), c_vp)
_sig("hc_plan_plain_db", _st, c_vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
     ctypes.c_uint32, c_u32p, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(CompressInfo))
_sig("hc_compress_batch", _st, c_vp, c_vp, c_vp, ctypes.POINTER(Query), ctypes.c_uint32, c_vp)
_sig("hc_graph_create", _st, c_vp, c_vp, c_vp, ctypes.POINTER(Query), ctypes.c_uint32, ctypes.POINTER(c_vp))
_sig("hc_graph_launch", _st, c_vp, c_vp)
_sig("hc_graph_nodes", _st, c_vp, ctypes.POINTER(ctypes.c_uint64))
_sig("hc_graph_destroy", None, c_vp)
_sig("hc_autotune", _st, c_vp, c_vp, c_vp, c_vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, c_vp,
     ctypes.POINTER(TuneReport), c_vp)
_sig("hc_tune_set", _st, c_vp, ctypes.c_uint32, ctypes.c_uint32)
_sig("hc_tune_get", _st, c_vp, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32))
_sig("hc_relin_keygen", _st, c_vp, c_vp, c_u8p, ctypes.POINTER(c_vp))
_sig("hc_mul", _st, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp)
_sig("hc_power", _st, c_vp, c_vp, c_vp, ctypes.c_uint32, c_vp, c_vp)
_sig("hc_match", _st, c_vp, c_vp, c_vp, c_vp, ctypes.c_uint64, c_vp, c_vp)
_sig("hc_compress_generic", _st, c_vp, c_vp, c_vp, c_vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
     ctypes.c_uint32, c_vp, ctypes.POINTER(CompressInfo), c_vp)
_sig("hc_decrypt", _st, c_vp, c_vp, c_u64p, ctypes.c_uint32, c_u32p)
_sig("hc_decompress", _st, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
     c_u32p, c_u32p, c_u64p, c_u32p, c_u32p)
_sig("hc_ntt", _st, c_vp, c_vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, c_vp)
_sig("hc_rotate", _st, c_vp, c_vp, ctypes.c_uint32, c_vp, c_vp, c_vp)
_sig("hc_rotate_level", _st, c_vp, c_vp, ctypes.c_uint32, ctypes.c_uint32, c_vp, c_vp, c_vp)
_sig("hc_rotate_level_noalloc", _st, c_vp, c_vp, ctypes.c_uint32, ctypes.c_uint32, c_vp, c_vp, c_vp)
_sig("hc_mod_switch", _st, c_vp, c_vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, c_vp, c_vp)
_sig("hc_rotate_hoisted", _st, c_vp, c_vp, c_u32p, ctypes.c_uint32, c_vp, c_vp, c_vp)
_sig("hc_mul_plain", _st, c_vp, c_vp, c_u32p, c_vp, c_vp)
_sig("hc_modup", _st, c_vp, c_vp, ctypes.c_uint32, c_vp, c_vp)
_sig("hc_moddown", _st, c_vp, c_vp, c_vp, c_vp)
_sig("hc_sample", _st, c_vp, ctypes.c_int, c_u8p, ctypes.c_char_p, ctypes.c_uint64, ctypes.c_uint32,
     c_vp, c_vp)
_sig("hc_encode_diagonal", _st, c_vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
     ctypes.c_uint32, ctypes.c_uint32, c_vp, c_vp)
_sig("hc_export_sk", _st, c_vp, c_vp, c_i64p)
_sig("hc_export_pk", _st, c_vp, c_vp, c_u64p)
_sig("hc_export_gk", _st, c_vp, c_vp, ctypes.c_uint32, c_u64p)
_sig("hc_timing_enable", _st, c_vp, ctypes.c_int)
_sig("hc_timing_read", _st, c_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
     ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double))
_sig("hc_probe_mul32_rate", _st, c_vp, ctypes.c_double, ctypes.POINTER(ctypes.c_double))
_sig("hc_probe_copy", _st, c_vp, ctypes.c_uint64)
_sig("hc_probe_stream", _st, c_vp, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(ctypes.c_double))
_sig("hc_diag_prepare", _st, c_vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
     ctypes.POINTER(ctypes.c_uint64))
_sig("hc_diag_release", None, c_vp)
_sig("hc_diag_layout", _st, c_vp, ctypes.c_int)
_sig("hc_server_create", _st, c_vp, c_vp, c_vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32,
     ctypes.c_uint32, ctypes.POINTER(c_vp))
_sig("hc_server_submit", _st, c_vp, c_vp, ctypes.c_uint64, ctypes.c_uint32, c_vp, c_vp,
     ctypes.POINTER(ctypes.c_uint64))
_sig("hc_server_poll", _st, c_vp, ctypes.POINTER(ServerResult), ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32),
     ctypes.c_double)
_sig("hc_server_stats_get", _st, c_vp, ctypes.POINTER(ServerStats))
_sig("hc_server_destroy", None, c_vp)

KT_NTT_FWD, KT_NTT_INV, KT_KS_INNER, KT_DIAG_MAC, KT_MODUP, KT_CONV_FUSED = 0, 1, 2, 3, 4, 5
KT_NAMES = {KT_NTT_FWD: "ntt_forward", KT_NTT_INV: "ntt_inverse", KT_KS_INNER: "keyswitch_inner",
            KT_DIAG_MAC: "diag_mac", KT_MODUP: "modup", KT_CONV_FUSED: "conv_fused"}

EXPORTED = [
    "hc_status_str", "hc_context_create", "hc_context_destroy", "hc_context_primes", "hc_context_trim",
    "hc_keygen",
    "hc_sk_destroy", "hc_pk_destroy", "hc_galois_keygen", "hc_gk_destroy", "hc_plan",
    "hc_db_upload", "hc_db_destroy", "hc_encrypt", "hc_compress", "hc_compress_batch",
    "hc_compress_plain_db", "hc_plan_plain_db",
    "hc_decrypt", "hc_decompress", "hc_ntt", "hc_rotate", "hc_rotate_level", "hc_rotate_level_noalloc", "hc_mod_switch",
    "hc_rotate_hoisted", "hc_mul_plain",
    "hc_modup", "hc_moddown", "hc_sample", "hc_encode_diagonal", "hc_export_sk", "hc_export_pk",
    "hc_export_gk", "hc_timing_enable", "hc_timing_read", "hc_probe_mul32_rate", "hc_probe_copy", "hc_probe_stream",
    "hc_graph_create", "hc_graph_launch", "hc_graph_nodes", "hc_graph_destroy",
    "hc_autotune", "hc_tune_set", "hc_tune_get",
    "hc_relin_keygen", "hc_mul", "hc_power", "hc_match", "hc_compress_generic",
    "hc_diag_prepare", "hc_diag_release", "hc_diag_layout", "hc_server_create", "hc_server_submit", "hc_server_poll",
    "hc_server_stats_get", "hc_server_destroy",
]


def lib():
    return _lib


def _check(st, what):
    if st != HC_OK:
        raise HcError(st, what)


def _u8(b):
    assert len(b) == 32
    return (ctypes.c_uint8 * 32).from_buffer_copy(b)


def _np_ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _dev(t, words=None, what="buffer"):
    """Device address of an int64 CUDA tensor; with `words`, the tensor must hold at
    least that many 64-bit words (else HC_EINVAL is raised before any library call)."""
    import torch
    assert t.is_cuda and t.dtype == torch.int64 and t.is_contiguous()
    if words is not None and t.numel() < words:
        raise HcError(HC_EINVAL, "%s holds %d words, %d needed" % (what, t.numel(), words))
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """A library context for one ring/modulus setting on one device."""

    def __init__(self, log_n, p, L, q_bits, K, p_bits, device=0):
        self.params = Params(log_n, p, L, q_bits, K, p_bits)
        self.n = 1 << log_n
        self.nh = self.n // 2
        self.p, self.L, self.K = p, L, K
        self.nq = L + K
        self.dnum = L // K
        self.device = device
        h = c_vp()
        _check(_lib.hc_context_create(ctypes.byref(self.params), device, ctypes.byref(h)),
               "hc_context_create")
        self.h = h
        pr = np.zeros(L + K, dtype=np.uint64)
        _check(_lib.hc_context_primes(self.h, _np_ptr(pr, ctypes.c_uint64)), "hc_context_primes")
        self.primes = [int(x) for x in pr]

    def close(self):
        if self.h:
            _lib.hc_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- torch helpers
    def trim(self):
        """Free the per-call device workspace (it grows again on demand)."""
        _lib.hc_context_trim(self.h)

    def ct_tensor(self, count=1):
        import torch
        return torch.empty((count, 2, self.L, self.n), dtype=torch.int64, device="cuda:%d" % self.device)

    # ---- keys
    def keygen(self, seed):
        sk, pk = c_vp(), c_vp()
        _check(_lib.hc_keygen(self.h, _u8(seed), ctypes.byref(sk), ctypes.byref(pk)), "hc_keygen")
        return SecretKey(self, sk), PublicKey(self, pk)

    def galois_keygen(self, sk, elements, seed):
        arr = np.asarray(elements, dtype=np.uint32)
        gk = c_vp()
        _check(_lib.hc_galois_keygen(self.h, sk.h, _np_ptr(arr, ctypes.c_uint32), len(arr), _u8(seed),
                                     ctypes.byref(gk)), "hc_galois_keygen")
        return GaloisKeys(self, gk, [int(x) for x in arr])

    def relin_keygen(self, sk, seed):
        rk = c_vp()
        _check(_lib.hc_relin_keygen(self.h, sk.h, _u8(seed), ctypes.byref(rk)), "hc_relin_keygen")
        return GaloisKeys(self, rk, [1])

    def mul(self, rk, a, b, out=None, stream=None):
        out = self.ct_tensor(1)[0] if out is None else out
        w = 2 * self.L * self.n
        _check(_lib.hc_mul(self.h, rk.h, _dev(a, w, "ct_a"), _dev(b, w, "ct_b"), _dev(out, w, "out"),
                           _stream(stream)), "hc_mul")
        return out

    def power(self, rk, ct, exponent, out=None, stream=None):
        out = self.ct_tensor(1)[0] if out is None else out
        w = 2 * self.L * self.n
        _check(_lib.hc_power(self.h, rk.h, _dev(ct, w, "ct_in"), exponent, _dev(out, w, "out"), _stream(stream)),
               "hc_power")
        return out

    def match(self, rk, keys_db, ct_x, N, out=None, stream=None):
        """Index-vector ciphertexts [ceil(N/n)][2][L][n] of [k_r = x] (keys: column 0 of keys_db)."""
        out = self.ct_tensor(-(-int(N) // self.n)) if out is None else out
        _check(_lib.hc_match(self.h, rk.h, keys_db.h, _dev(ct_x, 2 * self.L * self.n, "ct_x"), N,
                             _dev(out, self.ct_words(N), "ct_v"), _stream(stream)), "hc_match")
        return out

    def compress_generic(self, gk, rk, ct_d, N, t_bound, out=None, stream=None, comp_level=0, out_level=0):
        """Alg. 5: Power_{p-1} of d, then Comp of (v, d); returns (out, info)."""
        out = self.ct_tensor(1)[0] if out is None else out
        info = CompressInfo()
        _check(_lib.hc_compress_generic(self.h, gk.h, rk.h, _dev(ct_d, self.ct_words(N), "ct_d"), N, t_bound,
                                        comp_level, out_level, _dev(out, 2 * self.L * self.n, "out"),
                                        ctypes.byref(info), _stream(stream)), "hc_compress_generic")
        return out, info.as_dict()

    def plan(self, N, ncol, t_bound, comp_level=0, out_level=0):
        cnt = ctypes.c_uint32(0)
        info = CompressInfo()
        st = _lib.hc_plan(self.h, N, ncol, t_bound, comp_level, out_level, None, ctypes.byref(cnt),
                          ctypes.byref(info))
        if st not in (HC_OK, HC_EINVAL) or (st == HC_EINVAL and cnt.value == 0):
            _check(st, "hc_plan")
        arr = np.zeros(max(cnt.value, 1), dtype=np.uint32)
        cap = ctypes.c_uint32(len(arr))
        _check(_lib.hc_plan(self.h, N, ncol, t_bound, comp_level, out_level, _np_ptr(arr, ctypes.c_uint32),
                            ctypes.byref(cap), ctypes.byref(info)), "hc_plan")
        return [int(x) for x in arr[:cap.value]], info.as_dict()

    def plan_plain_db(self, N, ncol, t_bound, comp_level=0, out_level=0):
        """Key set and counts of the unencrypted-database form."""
        cnt = ctypes.c_uint32(0)
        info = CompressInfo()
        st = _lib.hc_plan_plain_db(self.h, N, ncol, t_bound, comp_level, out_level, None, ctypes.byref(cnt),
                                   ctypes.byref(info))
        if st not in (HC_OK, HC_EINVAL) or (st == HC_EINVAL and cnt.value == 0):
            _check(st, "hc_plan_plain_db")
        arr = np.zeros(max(cnt.value, 1), dtype=np.uint32)
        cap = ctypes.c_uint32(len(arr))
        _check(_lib.hc_plan_plain_db(self.h, N, ncol, t_bound, comp_level, out_level,
                                     _np_ptr(arr, ctypes.c_uint32), ctypes.byref(cap), ctypes.byref(info)),
               "hc_plan_plain_db")
        return [int(x) for x in arr[:cap.value]], info.as_dict()

    def compress_plain_db(self, gk, db, ct_v, N, t_bound, out=None, stream=None, comp_level=0, out_level=0):
        """The unencrypted-database form: (out buffer, info), like compress()."""
        out = self.ct_tensor(1)[0] if out is None else out
        info = CompressInfo()
        _check(_lib.hc_compress_plain_db(self.h, gk.h, db.h if db is not None else None,
                                         _dev(ct_v, self.ct_words(N), "ct_v"), N, t_bound, comp_level, out_level,
                                         _dev(out, 2 * self.L * self.n, "out"), ctypes.byref(info),
                                         _stream(stream)), "hc_compress_plain_db")
        return out, info.as_dict()

    def diag_prepare(self, N, ncol, t_bound, comp_level=0):
        """Encode and keep resident the diagonals these compressions use; returns the
        device bytes held by all resident tables."""
        b = ctypes.c_uint64(0)
        _check(_lib.hc_diag_prepare(self.h, N, ncol, t_bound, comp_level, ctypes.byref(b)), "hc_diag_prepare")
        return int(b.value)

    def diag_release(self):
        _lib.hc_diag_release(self.h)

    def diag_layout(self, layout):
        """Layout of the tables later diag_prepare calls build: DIAG_LAYOUT_AUTO (matrix-core
        digits where a class fits them) or DIAG_LAYOUT_SPLIT (split words everywhere)."""
        _check(_lib.hc_diag_layout(self.h, int(layout)), "hc_diag_layout")

    def db_upload(self, cols):
        cols = np.ascontiguousarray(cols, dtype=np.uint32)
        ncol, N = (cols.shape[0], cols.shape[1]) if cols.ndim == 2 else (0, int(cols))
        db = c_vp()
        _check(_lib.hc_db_upload(self.h, _np_ptr(cols, ctypes.c_uint32), ncol, N, ctypes.byref(db)),
               "hc_db_upload")
        return Database(self, db, ncol, N)

    def db_empty(self, N):
        db = c_vp()
        _check(_lib.hc_db_upload(self.h, None, 0, N, ctypes.byref(db)), "hc_db_upload")
        return Database(self, db, 0, N)

    # ---- encryption / compression
    def encrypt(self, pk, slots, seed, out=None, stream=None):
        sl = np.ascontiguousarray(slots, dtype=np.uint32).reshape(2, self.nh)
        out = self.ct_tensor(1)[0] if out is None else out
        _check(_lib.hc_encrypt(self.h, pk.h, _np_ptr(sl, ctypes.c_uint32), _u8(seed), _dev(out),
                               _stream(stream)), "hc_encrypt")
        return out

    def ct_words(self, N):
        """64-bit words of the index-vector ciphertexts of N records, [ceil(N/n)][2][L][n]."""
        return -(-int(N) // self.n) * 2 * self.L * self.n

    def compress(self, gk, db, ct_v, N, t_bound, out=None, stream=None, comp_level=0, out_level=0):
        """Returns (out buffer, info); output() extracts the [2][level][n] ciphertext."""
        out = self.ct_tensor(1)[0] if out is None else out
        info = CompressInfo()
        _check(_lib.hc_compress(self.h, gk.h, db.h if db is not None else None,
                                _dev(ct_v, self.ct_words(N), "ct_v"), N, t_bound, comp_level, out_level,
                                _dev(out, 2 * self.L * self.n, "out"), ctypes.byref(info), _stream(stream)),
               "hc_compress")
        return out, info.as_dict()

    def output(self, out, info):
        """The [2][level][n] output ciphertext inside an hc_compress output buffer."""
        lvl = info["level"]
        return out.reshape(-1)[:2 * lvl * self.n].reshape(2, lvl, self.n)

    def compress_batch(self, gk, db, queries, stream=None, comp_level=0, out_level=0):
        """queries: list of (ct_v tensor, N, t_bound, out tensor)."""
        arr = (Query * len(queries))()
        infos = [CompressInfo() for _ in queries]
        for i, (ctv, N, t, out) in enumerate(queries):
            arr[i].ct_v = _dev(ctv, self.ct_words(N), "ct_v").value
            arr[i].N = N
            arr[i].t_bound = t
            arr[i].comp_level = comp_level
            arr[i].out_level = out_level
            arr[i].ct_out = _dev(out, 2 * self.L * self.n, "out").value
            arr[i].info = ctypes.pointer(infos[i])
        st = _lib.hc_compress_batch(self.h, gk.h, db.h if db is not None else None, arr, len(queries),
                                    _stream(stream))
        return st, [arr[i].status for i in range(len(queries))], [x.as_dict() for x in infos]

    def autotune(self, gk, db, ct_v, N, t_bound, comp_level=0, stream=None):
        """Pick the fastest bit-neutral kernel variants on this compression; returns the report."""
        rep = TuneReport()
        out = self.ct_tensor(1)[0]
        _check(_lib.hc_autotune(self.h, gk.h, db.h if db is not None else None, _dev(ct_v, self.ct_words(N), "ct_v"),
                                N, t_bound, comp_level, _dev(out), ctypes.byref(rep), _stream(stream)), "hc_autotune")
        return rep.as_dict()

    def tune_set(self, mac_variant, ntt_variant):
        _check(_lib.hc_tune_set(self.h, mac_variant, ntt_variant), "hc_tune_set")

    def tune_get(self):
        a, b = ctypes.c_uint32(0), ctypes.c_uint32(0)
        _check(_lib.hc_tune_get(self.h, ctypes.byref(a), ctypes.byref(b)), "hc_tune_get")
        return int(a.value), int(b.value)

    def graph(self, gk, db, queries, comp_level=0, out_level=0):
        """Capture hc_compress_batch over queries [(ct_v, N, t_bound, out)] into a Graph;
        each launch recomputes the answers of whatever the ct_v buffers hold."""
        arr = (Query * len(queries))()
        infos = [CompressInfo() for _ in queries]
        keep = []
        for i, (ctv, N, t, out) in enumerate(queries):
            arr[i].ct_v = _dev(ctv, self.ct_words(N), "ct_v").value
            arr[i].N = N
            arr[i].t_bound = t
            arr[i].comp_level = comp_level
            arr[i].out_level = out_level
            arr[i].ct_out = _dev(out, 2 * self.L * self.n, "out").value
            arr[i].info = ctypes.pointer(infos[i])
            keep.append((ctv, out))
        h = c_vp()
        _check(_lib.hc_graph_create(self.h, gk.h, db.h if db is not None else None, arr, len(queries),
                                    ctypes.byref(h)), "hc_graph_create")
        return Graph(self, h, keep, [x.as_dict() for x in infos])

    def decrypt(self, sk, ct_host):
        """ct_host: [2][level][n] (level inferred from the size)."""
        ct = np.ascontiguousarray(ct_host, dtype=np.uint64)
        level = ct.size // (2 * self.n)
        ct = ct.reshape(2, level, self.n)
        out = np.zeros((2, self.nh), dtype=np.uint32)
        _check(_lib.hc_decrypt(self.h, sk.h, _np_ptr(ct, ctypes.c_uint64), level,
                               _np_ptr(out, ctypes.c_uint32)), "hc_decrypt")
        return out

    # ---- kernel-level
    def ntt(self, data, limb_first, nlimbs, inverse=False, stream=None):
        count = data.numel() // (nlimbs * self.n)
        _check(_lib.hc_ntt(self.h, _dev(data), count, limb_first, nlimbs, 1 if inverse else 0,
                           _stream(stream)), "hc_ntt")

    def rotate(self, gk, element, ct_in, out=None, stream=None):
        out = self.ct_tensor(1)[0] if out is None else out
        w = 2 * self.L * self.n
        _check(_lib.hc_rotate(self.h, gk.h, element, _dev(ct_in, w, "ct_in"), _dev(out, w, "out"),
                              _stream(stream)), "hc_rotate")
        return out

    def rotate_level(self, gk, element, level, ct_in, out=None, stream=None):
        """Rotation of a [2][level][n] ciphertext with the key restricted to level primes."""
        import torch
        w = 2 * level * self.n
        out = torch.empty(w, dtype=torch.int64, device=ct_in.device) if out is None else out
        _check(_lib.hc_rotate_level(self.h, gk.h, element, level, _dev(ct_in, w, "ct_in"), _dev(out, w, "out"),
                                    _stream(stream)), "hc_rotate_level")
        return out

    def rotate_level_noalloc(self, gk, element, level, ct_in, out, stream=None):
        """hc_rotate_level through the allocation-free entry point (out is required:
        the call allocates nothing, so neither does this wrapper)."""
        w = 2 * level * self.n
        _check(_lib.hc_rotate_level_noalloc(self.h, gk.h, element, level, _dev(ct_in, w, "ct_in"),
                                            _dev(out, w, "out"), _stream(stream)), "hc_rotate_level_noalloc")
        return out

    def mod_switch(self, ct_in, level_in, level_out, count=1, out=None, stream=None):
        """Drop primes level_out..level_in-1 of `count` coefficient-domain ciphertexts."""
        import torch
        wo = count * 2 * level_out * self.n
        out = torch.empty(wo, dtype=torch.int64, device=ct_in.device) if out is None else out
        _check(_lib.hc_mod_switch(self.h, _dev(ct_in, count * 2 * level_in * self.n, "ct_in"), count, level_in,
                                  level_out, _dev(out, wo, "out"), _stream(stream)), "hc_mod_switch")
        return out

    def rotate_hoisted(self, gk, elements, ct_in, stream=None):
        arr = np.asarray(elements, dtype=np.uint32)
        out = self.ct_tensor(len(arr))
        _check(_lib.hc_rotate_hoisted(self.h, gk.h, _np_ptr(arr, ctypes.c_uint32), len(arr), _dev(ct_in),
                                      _dev(out), _stream(stream)), "hc_rotate_hoisted")
        return out

    def mul_plain(self, ct_in, slots, out=None, stream=None):
        sl = np.ascontiguousarray(slots, dtype=np.uint32).reshape(2, self.nh)
        out = self.ct_tensor(1)[0] if out is None else out
        _check(_lib.hc_mul_plain(self.h, _dev(ct_in), _np_ptr(sl, ctypes.c_uint32), _dev(out),
                                 _stream(stream)), "hc_mul_plain")
        return out

    def modup(self, x, digit, out, stream=None):
        _check(_lib.hc_modup(self.h, _dev(x), digit, _dev(out), _stream(stream)), "hc_modup")

    def moddown(self, T, out, stream=None):
        _check(_lib.hc_moddown(self.h, _dev(T), _dev(out), _stream(stream)), "hc_moddown")

    def sample(self, kind, seed, tag, obj, limb, out, stream=None):
        _check(_lib.hc_sample(self.h, kind, _u8(seed), tag.encode(), obj, limb, _dev(out), _stream(stream)),
               "hc_sample")

    def encode_diagonal(self, s, B, beta, gi, b, out, stream=None):
        _check(_lib.hc_encode_diagonal(self.h, s, B, beta, gi, b, _dev(out), _stream(stream)),
               "hc_encode_diagonal")

    def timing(self, enable):
        _check(_lib.hc_timing_enable(self.h, 1 if enable else 0), "hc_timing_enable")

    def timing_read(self, kind):
        ms, by, op = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        cnt = ctypes.c_uint64()
        _check(_lib.hc_timing_read(self.h, kind, ctypes.byref(ms), ctypes.byref(cnt), ctypes.byref(by),
                                   ctypes.byref(op)), "hc_timing_read")
        return dict(ms=ms.value, launches=cnt.value, bytes=by.value, ops=op.value)

    def probe_mul32_rate(self, ms=50.0):
        r = ctypes.c_double()
        _check(_lib.hc_probe_mul32_rate(self.h, ms, ctypes.byref(r)), "hc_probe_mul32_rate")
        return r.value

    def probe_copy(self, nbytes):
        _check(_lib.hc_probe_copy(self.h, int(nbytes)), "hc_probe_copy")

    def probe_stream(self, read_bytes, write_bytes, reps=3):
        """Mean ms per launch of the read/write stream probe (hc_probe_stream)."""
        ms = ctypes.c_double(0)
        _check(_lib.hc_probe_stream(self.h, int(read_bytes), int(write_bytes), int(reps), ctypes.byref(ms)),
               "hc_probe_stream")
        return ms.value

    def export_sk(self, sk):
        out = np.zeros(self.n, dtype=np.int64)
        _check(_lib.hc_export_sk(self.h, sk.h, _np_ptr(out, ctypes.c_int64)), "hc_export_sk")
        return out

    def export_pk(self, pk):
        out = np.zeros((2, self.L, self.n), dtype=np.uint64)
        _check(_lib.hc_export_pk(self.h, pk.h, _np_ptr(out, ctypes.c_uint64)), "hc_export_pk")
        return out

    def export_gk(self, gk, element):
        out = np.zeros((self.dnum, 2, self.nq, self.n), dtype=np.uint64)
        _check(_lib.hc_export_gk(self.h, gk.h, element, _np_ptr(out, ctypes.c_uint64)), "hc_export_gk")
        return out


def decompress(p, N_group, s, w, es):
    """Decomp for one group: (indices 1-based ascending, values [ncols][count])."""
    w = np.ascontiguousarray(w, dtype=np.uint32)
    es = np.ascontiguousarray(es, dtype=np.uint32).reshape(-1, s) if len(es) else np.zeros((0, s), np.uint32)
    ncols = es.shape[0]
    idx = np.zeros(s, dtype=np.uint64)
    vals = np.zeros((max(ncols, 1), s), dtype=np.uint32)
    cnt = ctypes.c_uint32(0)
    _check(_lib.hc_decompress(p, N_group, s, ncols, _np_ptr(w, ctypes.c_uint32),
                              _np_ptr(es, ctypes.c_uint32) if ncols else None, _np_ptr(idx, ctypes.c_uint64),
                              _np_ptr(vals, ctypes.c_uint32) if ncols else None, ctypes.byref(cnt)),
           "hc_decompress")
    l = cnt.value
    return [int(x) for x in idx[:l]], [[int(x) for x in vals[c, :l]] for c in range(ncols)]


class _Handle:
    _destroy = None

    def __init__(self, ctx, h):
        self.ctx, self.h = ctx, h

    def close(self):
        if self.h and self.ctx.h:
            getattr(_lib, self._destroy)(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SecretKey(_Handle):
    _destroy = "hc_sk_destroy"


class PublicKey(_Handle):
    _destroy = "hc_pk_destroy"


class GaloisKeys(_Handle):
    _destroy = "hc_gk_destroy"

    def __init__(self, ctx, h, elements):
        super().__init__(ctx, h)
        self.elements = elements


class Database(_Handle):
    _destroy = "hc_db_destroy"

    def __init__(self, ctx, h, ncol, N):
        super().__init__(ctx, h)
        self.ncol, self.N = ncol, N


class Graph(_Handle):
    """A captured batch of compressions (hc_graph_*); keeps its buffers alive."""
    _destroy = "hc_graph_destroy"

    def __init__(self, ctx, h, buffers, infos):
        super().__init__(ctx, h)
        self.buffers, self.infos = buffers, infos

    def launch(self, stream=None):
        _check(_lib.hc_graph_launch(self.h, _stream(stream)), "hc_graph_launch")

    def nodes(self):
        n = ctypes.c_uint64(0)
        _check(_lib.hc_graph_nodes(self.h, ctypes.byref(n)), "hc_graph_nodes")
        return int(n.value)


class Server:
    """Serving loop (hc_server_*): submit queries as they arrive, poll completions.
    Keeps every submitted request's device tensors alive until it is polled."""

    def __init__(self, ctx, gk, db, comp_level=0, lane_bytes=8 << 30, lanes=2, max_batch=16, out_level=0):
        self.ctx, self.gk, self.db = ctx, gk, db
        h = c_vp()
        _check(_lib.hc_server_create(ctx.h, gk.h, db.h if db is not None else None, comp_level, out_level,
                                     lane_bytes, lanes, max_batch, ctypes.byref(h)), "hc_server_create")
        self.h = h
        self._live = {}

    def submit(self, ct_v, N, t_bound, out, stream=None):
        """ct_v may still be in flight on `stream` (torch's current stream by default)."""
        rid = ctypes.c_uint64(0)
        c = self.ctx
        _check(_lib.hc_server_submit(self.h, _dev(ct_v, c.ct_words(N), "ct_v"), N, t_bound,
                                     _dev(out, 2 * c.L * c.n, "out"), _stream(stream), ctypes.byref(rid)),
               "hc_server_submit")
        self._live[rid.value] = (ct_v, out)
        return rid.value

    def poll(self, cap=64, timeout_ms=0.0):
        arr = (ServerResult * cap)()
        cnt = ctypes.c_uint32(0)
        _check(_lib.hc_server_poll(self.h, arr, cap, ctypes.byref(cnt), float(timeout_ms)), "hc_server_poll")
        res = []
        for i in range(cnt.value):
            r = arr[i]
            self._live.pop(r.id, None)
            res.append({"id": r.id, "status": r.status, "submit_ns": r.submit_ns, "start_ns": r.start_ns,
                        "done_ns": r.done_ns, "batch_size": r.batch_size, "info": r.info.as_dict()})
        return res

    def stats(self):
        st = ServerStats()
        _check(_lib.hc_server_stats_get(self.h, ctypes.byref(st)), "hc_server_stats_get")
        return {f: getattr(st, f) for f, _ in st._fields_}

    def close(self):
        if self.h:
            _lib.hc_server_destroy(self.h)
            self.h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

