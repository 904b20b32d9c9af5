"""Python binding of the gfx950 Paillier histogram library (include/he.h).

Argument marshalling only: every step runs in the HIP kernels of
``libhe_mi355x.so``.  Device buffers are torch tensors on a ROCm device;
uint32 limb arrays travel as int32 tensors (same bits).  Calls enqueue on the
current torch stream unless a stream is passed.  There is no CPU fallback: if
the shared library is missing, importing this module raises.
"""
from __future__ import annotations

import collections
import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhe_mi355x.so")

HE_OK = 0
HE_ERR_ARG, HE_ERR_KEY, HE_ERR_NOPRIV, HE_ERR_RANGE, HE_ERR_OOM, HE_ERR_DEVICE = -1, -2, -3, -4, -5, -6
HE_FORM_CANONICAL, HE_FORM_MONT = 0, 1

EXPORTED = (
    "he_keygen", "he_key_import", "he_key_export", "he_key_bits", "he_key_has_private",
    "he_key_free", "he_encode", "he_encrypt", "he_encrypt_public", "he_to_mont", "he_from_mont",
    "he_hist_aggregate", "he_hist_aggregate_ex", "he_decrypt", "he_probe_int_mul", "he_last_error",
    "he_hist_autotune", "he_hist_plan_create", "he_hist_plan_launch", "he_hist_plan_free",
    "he_obfuscators", "he_encrypt_obfuscated", "he_hist_subtract", "he_split_find",
    "he_hist_aggregate_counted", "he_ct_mul", "he_pack_slots", "he_pack", "he_decrypt_packed",
    "he_decrypt_noalloc", "he_key_set_constant_time", "he_crt_autotune", "he_crt_set_shape",
)


class HEError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"he error {code}: {msg}")
        self.code = code


def _load() -> ctypes.CDLL:
    if not os.path.exists(_LIB_PATH):
        raise ImportError(
            f"{_LIB_PATH} is missing: build it with `python -m paper_2504_03909_amd.build` "
            "(there is no CPU fallback)")
    return ctypes.CDLL(_LIB_PATH)


_lib = _load()
_vp, _u32, _u64, _i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int


class HistJob(ctypes.Structure):
    _fields_ = [("sample_idx", _vp), ("n_samples", _u64), ("bins", _vp), ("bins_ld", _u64),
                ("n_features", _u32), ("n_bins", _u32), ("hist", _vp), ("n_bad", _vp)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_keygen = _sig("he_keygen", _i32, [_u32, _u64, ctypes.POINTER(_vp)])
_key_import = _sig("he_key_import", _i32, [_u32, _vp, _vp, ctypes.POINTER(_vp)])
_key_export = _sig("he_key_export", _i32, [_vp, _vp, _vp, _vp])
_key_bits = _sig("he_key_bits", _u32, [_vp])
_key_priv = _sig("he_key_has_private", _i32, [_vp])
_key_free = _sig("he_key_free", None, [_vp])
_key_ct = _sig("he_key_set_constant_time", _i32, [_vp, _i32])
_encode = _sig("he_encode", _i32, [_vp, _u64, _u32, _vp, _vp, _vp])
_encrypt = _sig("he_encrypt", _i32, [_vp, _vp, _u64, _vp, _u64, _u64, _vp, _vp])
_encrypt_pub = _sig("he_encrypt_public", _i32, [_vp, _vp, _u64, _vp, _u64, _u64, _vp, _vp])
_obf = _sig("he_obfuscators", _i32, [_vp, _u64, _vp, _u64, _u64, _vp, _vp])
_enc_obf = _sig("he_encrypt_obfuscated", _i32, [_vp, _vp, _u64, _vp, _vp, _vp])
_f64 = ctypes.c_double
_split = _sig("he_split_find", _i32, [_vp, _vp, _u32, _u32, _u32, _u32, _f64, _f64, _f64, _vp, _vp, _vp, _vp])
_pack_slots = _sig("he_pack_slots", _u32, [_vp, _u64])
_pack = _sig("he_pack", _i32, [_vp, _vp, _u64, _u32, _vp, _vp])
_dec_packed = _sig("he_decrypt_packed", _i32, [_vp, _vp, _u64, _u32, _vp, _vp, _vp])
_ct_mul = _sig("he_ct_mul", _i32, [_vp, _vp, _vp, _u64, _vp, _vp])
_sub = _sig("he_hist_subtract", _i32, [_vp, _vp, _vp, _u64, _u32, _vp, _vp, _vp])
_to_mont = _sig("he_to_mont", _i32, [_vp, _vp, _u64, _vp, _vp])
_from_mont = _sig("he_from_mont", _i32, [_vp, _vp, _u64, _vp, _vp])
_hist_counted = _sig("he_hist_aggregate_counted", _i32, [_vp, _vp, _u64, _i32, ctypes.POINTER(HistJob), _u32,
                                                         _u32, _u32, _u32, _u32, _vp, _vp])
_hist = _sig("he_hist_aggregate_ex", _i32, [_vp, _vp, _u64, _i32, ctypes.POINTER(HistJob), _u32, _u32, _vp])
_decrypt = _sig("he_decrypt", _i32, [_vp, _vp, _u64, _vp, _vp, _vp, _vp])
_decrypt_noalloc = _sig("he_decrypt_noalloc", _i32, [_vp, _vp, _u64, _vp, _vp, _vp, _vp])
_probe = _sig("he_probe_int_mul", _i32, [_u64, _u32, ctypes.POINTER(_u64), _vp])
_last_error = _sig("he_last_error", ctypes.c_char_p, [])
_autotune = _sig("he_hist_autotune", _i32, [_vp, _vp, _u64, _i32, ctypes.POINTER(HistJob), _u32,
                                            ctypes.POINTER(_u32), ctypes.POINTER(_u32), ctypes.POINTER(_u32),
                                            ctypes.POINTER(_u32), ctypes.POINTER(ctypes.c_float), _vp])
_crt_autotune = _sig("he_crt_autotune", _i32, [_vp, _u64, _u64, ctypes.POINTER(_u32), ctypes.POINTER(ctypes.c_float),
                                               _vp])
_crt_set_shape = _sig("he_crt_set_shape", _i32, [_vp, _u32, _u64, _u32, _u32, _u32])
_plan_create = _sig("he_hist_plan_create", _i32, [_vp, _vp, _u64, _i32, ctypes.POINTER(HistJob), _u32, _u32,
                                                  _u32, ctypes.POINTER(_vp)])
_plan_launch = _sig("he_hist_plan_launch", _i32, [_vp, _vp])
_plan_free = _sig("he_hist_plan_free", None, [_vp])


def _check(rc: int) -> None:
    if rc != HE_OK:
        raise HEError(rc, (_last_error() or b"").decode())


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


# ----------------------------------------------------------- limb conversion
def ints_to_limbs(values: Sequence[int], n_limbs: int) -> np.ndarray:
    """Python ints -> int32 array [len, n_limbs] of little-endian 32-bit limbs."""
    out = np.zeros((len(values), n_limbs), dtype=np.uint32)
    nbytes = 4 * n_limbs
    for i, v in enumerate(values):
        out[i] = np.frombuffer(int(v).to_bytes(nbytes, "little"), dtype=np.uint32)
    return out.view(np.int32)


def limbs_to_ints(arr) -> List[int]:
    """int32/uint32 array [..., n_limbs] -> flat list of Python ints."""
    a = np.ascontiguousarray(np.asarray(arr).view(np.uint32))
    a = a.reshape(-1, a.shape[-1])
    return [int.from_bytes(row.tobytes(), "little") for row in a]


# -------------------------------------------------------------------- keys
class Key:
    """A Paillier key resident on the current device (n, n^2, p, q, p^2, q^2
    Montgomery constants and CRT constants)."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)

    @classmethod
    def generate(cls, n_bits: int, seed: int) -> "Key":
        h = _vp()
        _check(_keygen(n_bits, seed, ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def from_primes(cls, n_bits: int, p: int, q: int) -> "Key":
        half = n_bits // 64
        pa = np.frombuffer(int(p).to_bytes(4 * half, "little"), dtype=np.uint32).copy()
        qa = np.frombuffer(int(q).to_bytes(4 * half, "little"), dtype=np.uint32).copy()
        h = _vp()
        _check(_key_import(n_bits, pa.ctypes.data, qa.ctypes.data, ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def public(cls, n_bits: int, n: int) -> "Key":
        na = np.frombuffer(int(n).to_bytes(n_bits // 8, "little"), dtype=np.uint32).copy()
        h = _vp()
        _check(_key_import(n_bits, na.ctypes.data, None, ctypes.byref(h)))
        return cls(h.value)

    @property
    def handle(self):
        return self._h

    @property
    def bits(self) -> int:
        return int(_key_bits(self._h))

    @property
    def limbs(self) -> int:
        """Limbs of n (a ciphertext has 2 * limbs)."""
        return self.bits // 32

    @property
    def has_private(self) -> bool:
        return bool(_key_priv(self._h))

    def set_constant_time(self, on: bool = True) -> None:
        """Private-key exponentiations read every window-table entry (addresses
        independent of the secret exponent digits); results are unchanged."""
        _check(_key_ct(self._h, 1 if on else 0))

    def export(self):
        L = self.limbs
        n = np.zeros(L, dtype=np.uint32)
        if self.has_private:
            p = np.zeros(L // 2, dtype=np.uint32)
            q = np.zeros(L // 2, dtype=np.uint32)
            _check(_key_export(self._h, n.ctypes.data, p.ctypes.data, q.ctypes.data))
            return (int.from_bytes(n.tobytes(), "little"), int.from_bytes(p.tobytes(), "little"),
                    int.from_bytes(q.tobytes(), "little"))
        _check(_key_export(self._h, n.ctypes.data, None, None))
        return int.from_bytes(n.tobytes(), "little"), None, None

    def close(self):
        if self._h and self._h.value:
            _key_free(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ calls
def encode(x: torch.Tensor, frac_bits: int = 32, stream=None, n_bad: Optional[torch.Tensor] = None) -> torch.Tensor:
    """rint(x * 2^frac_bits) as int64 (device)."""
    assert x.dtype == torch.float64
    m = torch.empty(x.shape, dtype=torch.int64, device=x.device)
    _check(_encode(_ptr(x), x.numel(), frac_bits, _ptr(m), _ptr(n_bad), _stream(stream)))
    return m


def encrypt(key: Key, m: torch.Tensor, r: Optional[torch.Tensor] = None, seed: int = 0,
            offset: int = 0, public: bool = False, out: Optional[torch.Tensor] = None,
            stream=None) -> torch.Tensor:
    """Ciphertexts of the int64 plaintexts m (any shape) -> int32 [..., 2L]."""
    assert m.dtype == torch.int64
    m = m.contiguous()
    count = m.numel()
    L = key.limbs
    if r is not None:
        assert r.dtype == torch.int32 and r.shape[-1] == L and r.numel() == count * L
    if out is None:
        out = torch.empty((*m.shape, 2 * L), dtype=torch.int32, device=m.device)
    fn = _encrypt_pub if public else _encrypt
    _check(fn(key.handle, _ptr(m), count, _ptr(r), seed, offset, _ptr(out), _stream(stream)))
    return out


def obfuscators(key: Key, count: int, r: Optional[torch.Tensor] = None, seed: int = 0, offset: int = 0,
                out: Optional[torch.Tensor] = None, stream=None, device="cuda") -> torch.Tensor:
    """r_i^n mod n^2 for the same r as encrypt(seed=..., offset=...) -> int32 [count, 2L]."""
    if out is None:
        out = torch.empty((count, 2 * key.limbs), dtype=torch.int32, device=device)
    assert out.is_contiguous() and out.numel() == count * 2 * key.limbs
    _check(_obf(key.handle, count, _ptr(r), seed, offset, _ptr(out), _stream(stream)))
    return out


def encrypt_obfuscated(key: Key, m: torch.Tensor, rho: torch.Tensor, out: Optional[torch.Tensor] = None,
                       stream=None) -> torch.Tensor:
    """(1 + m n) rho mod n^2 -> int32 [..., 2L]; equals encrypt() with rho's r."""
    assert m.dtype == torch.int64 and rho.numel() == m.numel() * 2 * key.limbs
    m = m.contiguous()
    if out is None:
        out = torch.empty((*m.shape, 2 * key.limbs), dtype=torch.int32, device=m.device)
    _check(_enc_obf(key.handle, _ptr(m), m.numel(), _ptr(rho.contiguous()), _ptr(out), _stream(stream)))
    return out


def ct_mul(key: Key, a: torch.Tensor, b: torch.Tensor, out: Optional[torch.Tensor] = None,
           stream=None) -> torch.Tensor:
    """a * b mod n^2 elementwise (an encryption of m_a + m_b)."""
    assert a.shape == b.shape and a.shape[-1] == 2 * key.limbs
    a, b = a.contiguous(), b.contiguous()
    if out is None:
        out = torch.empty_like(a)
    _check(_ct_mul(key.handle, _ptr(a), _ptr(b), a.numel() // (2 * key.limbs), _ptr(out), _stream(stream)))
    return out


def rerandomize(key: Key, ct: torch.Tensor, seed: int, offset: int = 0, stream=None) -> torch.Tensor:
    """ct * E(0; r') mod n^2 with fresh r' from the seeded stream (public key
    suffices): same plaintexts, unlinkable ciphertexts."""
    count = ct.numel() // (2 * key.limbs)
    rho = obfuscators(key, count, seed=seed, offset=offset, stream=stream, device=ct.device)
    return ct_mul(key, ct, rho.view(ct.shape), out=torch.empty_like(ct), stream=stream)


def hist_subtract(key: Key, parent: torch.Tensor, child: torch.Tensor, out: Optional[torch.Tensor] = None,
                  batch: int = 0, n_bad: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """parent * child^-1 mod n^2 elementwise (an encryption of m_parent - m_child)."""
    assert parent.shape == child.shape and parent.shape[-1] == 2 * key.limbs
    parent, child = parent.contiguous(), child.contiguous()
    if out is None:
        out = torch.empty_like(parent)
    count = parent.numel() // (2 * key.limbs)
    _check(_sub(key.handle, _ptr(parent), _ptr(child), count, batch, _ptr(out), _ptr(n_bad), _stream(stream)))
    return out


def split_find(hist: torch.Tensor, minus: Optional[torch.Tensor] = None, frac_bits: int = 32,
               lam: float = 1.0, gamma: float = 0.0, min_child_weight: float = 1.0,
               derived: Optional[torch.Tensor] = None, per_feature: bool = False, stream=None):
    """Best splits from decrypted histograms hist int64 [nodes, F, B, 2]
    (the node histogram is hist - minus when minus is given).  Returns a dict
    of tensors: gain (float64), feature, bin (int32), g_left, h_left (int64)
    per node, and the same per (node, feature) under "per_feature"."""
    assert hist.dtype == torch.int64 and hist.dim() == 4 and hist.shape[-1] == 2
    nodes, F, B, _ = hist.shape
    hist = hist.contiguous()
    if minus is not None:
        assert minus.shape == hist.shape and minus.dtype == torch.int64
        minus = minus.contiguous()
    if derived is not None:
        assert derived.shape == hist.shape and derived.dtype == torch.int64 and derived.is_contiguous()
    out_node = torch.empty((nodes, 4), dtype=torch.int64, device=hist.device)   # 32-byte records
    out_feat = torch.empty((nodes, F, 4), dtype=torch.int64, device=hist.device) if per_feature else None
    _check(_split(_ptr(hist), _ptr(minus), nodes, F, B, frac_bits, lam, gamma, min_child_weight,
                  _ptr(derived), _ptr(out_feat), _ptr(out_node), _stream(stream)))

    def unpack(rec):
        fb = rec[..., 1:2].view(torch.int32)   # (feature, bin) int32 pair
        return {"gain": rec[..., 0].view(torch.float64), "feature": fb[..., 0], "bin": fb[..., 1],
                "g_left": rec[..., 2], "h_left": rec[..., 3]}
    res = unpack(out_node)
    if per_feature:
        res["per_feature"] = unpack(out_feat)
    return res


def to_mont(key: Key, ct: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    out = torch.empty_like(ct) if out is None else out
    _check(_to_mont(key.handle, _ptr(ct), ct.numel() // (2 * key.limbs), _ptr(out), _stream(stream)))
    return out


def from_mont(key: Key, ct: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    out = torch.empty_like(ct) if out is None else out
    _check(_from_mont(key.handle, _ptr(ct), ct.numel() // (2 * key.limbs), _ptr(out), _stream(stream)))
    return out


@dataclass
class Job:
    """One node's histogram job; tensors on the device."""
    sample_idx: torch.Tensor   # int32 [n] (row indices, uint32 bits)
    bins: torch.Tensor         # uint8 [F, ld]
    n_bins: int
    hist: Optional[torch.Tensor] = None  # int32 [F, B, 2, 2L], allocated if None
    n_bad: Optional[torch.Tensor] = None  # int32 [1]: skipped (sample, feature) pairs are added here

    def as_c(self, key: Key) -> HistJob:
        F, ld = self.bins.shape
        if self.hist is None:
            self.hist = torch.empty((F, self.n_bins, 2, 2 * key.limbs), dtype=torch.int32,
                                    device=self.bins.device)
        return HistJob(_ptr(self.sample_idx) if self.sample_idx.numel() else None,
                       self.sample_idx.numel(), _ptr(self.bins), ld, F, self.n_bins, _ptr(self.hist),
                       _ptr(self.n_bad))


def hist_aggregate(key: Key, ct: torch.Tensor, jobs: Sequence[Job], form: int = HE_FORM_CANONICAL,
                   chunk: int = 0, stream=None) -> List[torch.Tensor]:
    """Encrypted histograms of all jobs in one batch; ct is int32 [rows, 2, 2L]."""
    rows = ct.shape[0]
    arr = (HistJob * len(jobs))(*[j.as_c(key) for j in jobs])
    _check(_hist(key.handle, _ptr(ct), rows, form, arr, len(jobs), chunk, _stream(stream)))
    return [j.hist for j in jobs]


def hist_aggregate_counted(key: Key, ct: torch.Tensor, jobs: Sequence[Job], form: int = HE_FORM_CANONICAL,
                           chunk: int = 0, split: int = 2, lanes: int = 0, waves: int = 0, stream=None):
    """hist_aggregate at an explicit work shape (chunk, groups per item,
    lanes per ciphertext, waves per SIMD; 0 = default) plus the work
    counters: returns (hists, [real products, executed products, conversions
    out of Montgomery form])."""
    arr = (HistJob * len(jobs))(*[j.as_c(key) for j in jobs])
    cnt = torch.zeros(3, dtype=torch.int64, device=ct.device)
    _check(_hist_counted(key.handle, _ptr(ct), ct.shape[0], form, arr, len(jobs), chunk, split, lanes, waves,
                         _ptr(cnt), _stream(stream)))
    return [j.hist for j in jobs], cnt


HistTune = collections.namedtuple("HistTune", "chunk split lanes waves ms")


def hist_autotune(key: Key, ct: torch.Tensor, jobs: Sequence[Job], form: int = HE_FORM_CANONICAL,
                  stream=None) -> HistTune:
    """Times the batched aggregation of these jobs over the candidate work
    shapes; returns the fastest (chunk, split, lanes, waves, ms), which the
    library then uses for this shape class when chunk is 0."""
    arr = (HistJob * len(jobs))(*[j.as_c(key) for j in jobs])
    c, sp, ln, wv, ms = _u32(), _u32(), _u32(), _u32(), ctypes.c_float()
    _check(_autotune(key.handle, _ptr(ct), ct.shape[0], form, arr, len(jobs), ctypes.byref(c),
                     ctypes.byref(sp), ctypes.byref(ln), ctypes.byref(wv), ctypes.byref(ms), _stream(stream)))
    return HistTune(int(c.value), int(sp.value), int(ln.value), int(wv.value), float(ms.value))


PowTune = collections.namedtuple("PowTune", "lanes waves tail_lanes ms")


def crt_autotune(key: Key, enc_count: int, dec_count: int, stream=None):
    """Tunes the launch shapes of the private-key exponentiations for these
    counts (see he_crt_autotune); returns {kind: PowTune(lanes, waves,
    tail_lanes, ms)} for "mod_p", "lift" and "decrypt" (tail_lanes 0: one
    launch)."""
    choice = (_u32 * 9)()
    ms = (ctypes.c_float * 3)()
    _check(_crt_autotune(key.handle, enc_count, dec_count, choice, ms, _stream(stream)))
    return {name: PowTune(int(choice[3 * i]), int(choice[3 * i + 1]), int(choice[3 * i + 2]), float(ms[i]))
            for i, name in enumerate(("mod_p", "lift", "decrypt"))}


POW_KINDS = {"mod_p": 0, "lift": 1, "decrypt": 2, "public": 3}


def crt_set_shape(key: Key, kind: str, count: int, lanes: int, waves: int = 0, tail_lanes: int = 0) -> None:
    """Pins the launch shape of one exponentiation kind ("mod_p", "lift",
    "decrypt" or "public") for counts of count's size class (see
    he_crt_set_shape)."""
    _check(_crt_set_shape(key.handle, POW_KINDS[kind], count, lanes, waves, tail_lanes))


class HistPlan:
    """A batched aggregation captured into a HIP graph; launch() replays all
    of its kernels with one graph launch.  The tensors it was built from must
    stay alive (the plan keeps references)."""

    def __init__(self, key: Key, ct: torch.Tensor, jobs: Sequence[Job], form: int = HE_FORM_CANONICAL,
                 chunk: int = 0, split: int = 0):
        self._keep = (key, ct, list(jobs))
        arr = (HistJob * len(jobs))(*[j.as_c(key) for j in jobs])
        h = _vp()
        _check(_plan_create(key.handle, _ptr(ct), ct.shape[0], form, arr, len(jobs), chunk, split,
                            ctypes.byref(h)))
        self._h = h
        self.hists = [j.hist for j in jobs]

    def launch(self, stream=None):
        _check(_plan_launch(self._h, _stream(stream)))
        return self.hists

    def close(self):
        if self._h and self._h.value:
            _plan_free(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def decrypt(key: Key, ct: torch.Tensor, raw: bool = False, out: Optional[torch.Tensor] = None, stream=None):
    """Signed int64 plaintexts of ct (int32 [..., 2L]); optionally the raw
    plaintexts int32 [..., L] and the overflow count tensor."""
    count = ct.numel() // (2 * key.limbs)
    shape = ct.shape[:-1]
    if out is None:
        m = torch.empty(shape, dtype=torch.int64, device=ct.device)
    else:
        assert out.dtype == torch.int64 and out.is_contiguous() and out.numel() == count
        m = out
    rw = torch.empty((*shape, key.limbs), dtype=torch.int32, device=ct.device) if raw else None
    ovf = torch.zeros(1, dtype=torch.int32, device=ct.device)
    _check(_decrypt(key.handle, _ptr(ct.contiguous()), count, _ptr(m), _ptr(rw), _ptr(ovf), _stream(stream)))
    return m, rw, ovf


def decrypt_noalloc(key: Key, ct: torch.Tensor, m: torch.Tensor, raw: Optional[torch.Tensor] = None,
                    n_overflow: Optional[torch.Tensor] = None, stream=None) -> None:
    """he_decrypt into caller-provided outputs through the library's fixed
    device scratch (no device allocation by the library): m int64 [count],
    raw int32 [count, L] or None, n_overflow int32 [1] or None (not cleared)."""
    count = ct.numel() // (2 * key.limbs)
    assert ct.is_contiguous() and m.dtype == torch.int64 and m.is_contiguous() and m.numel() == count
    if raw is not None:
        assert raw.dtype == torch.int32 and raw.is_contiguous() and raw.numel() == count * key.limbs
    if n_overflow is not None:
        assert n_overflow.dtype == torch.int32 and n_overflow.numel() >= 1
    _check(_decrypt_noalloc(key.handle, _ptr(ct), count, _ptr(m), _ptr(raw), _ptr(n_overflow), _stream(stream)))


def pack_slots(key: Key, count: int) -> int:
    return int(_pack_slots(key.handle, count))


def pack(key: Key, ct: torch.Tensor, slots: int = 0, stream=None):
    """Folds ct (int32 [..., 2L], canonical) into ceil(count / slots)
    ciphertexts; slots 0 = the library's choice.  Returns (packed, slots)."""
    count = ct.numel() // (2 * key.limbs)
    slots = slots or pack_slots(key, count)
    packed = torch.empty(((count + slots - 1) // slots, 2 * key.limbs), dtype=torch.int32, device=ct.device)
    _check(_pack(key.handle, _ptr(ct.contiguous()), count, slots, _ptr(packed), _stream(stream)))
    return packed, slots


def decrypt_packed(key: Key, packed: torch.Tensor, count: int, slots: int, out: Optional[torch.Tensor] = None,
                   stream=None):
    """Signed int64 [count] values of packed ciphertexts, and the overflow count tensor."""
    if out is None:
        out = torch.empty(count, dtype=torch.int64, device=packed.device)
    assert out.dtype == torch.int64 and out.is_contiguous() and out.numel() == count
    ovf = torch.zeros(1, dtype=torch.int32, device=packed.device)
    _check(_dec_packed(key.handle, _ptr(packed.contiguous()), count, slots, _ptr(out), _ptr(ovf), _stream(stream)))
    return out, ovf


def probe_int_mul(iters: int, blocks: int, stream=None) -> int:
    prod = _u64()
    _check(_probe(iters, blocks, ctypes.byref(prod), _stream(stream)))
    return int(prod.value)


def library_path() -> str:
    return _LIB_PATH
