"""Python binding of the CKKS part of the library (include/he_ckks.h):
argument marshalling only, every step runs in the HIP kernels of
``libhe_mi355x.so``.  Polynomials travel as int32 tensors [count, 3, N]
(uint32 residues, same bits), ciphertexts as [count, 2, 3, N]."""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import he

_lib = he._lib
_vp, _u32, _u64, _i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int

EXPORTED = ("he_ckks_create", "he_ckks_free", "he_ckks_params", "he_ckks_encode", "he_ckks_encrypt",
            "he_ckks_add", "he_ckks_decrypt", "he_ckks_decode", "he_ckks_last_error")

_create = he._sig("he_ckks_create", _i32, [_u32, _u32, _u64, ctypes.POINTER(_vp)])
_free = he._sig("he_ckks_free", None, [_vp])
_params = he._sig("he_ckks_params", _i32, [_vp, ctypes.POINTER(_u32), _vp, ctypes.POINTER(_u32)])
_encode = he._sig("he_ckks_encode", _i32, [_vp, _vp, _u64, _u32, _vp, _vp])
_encrypt = he._sig("he_ckks_encrypt", _i32, [_vp, _vp, _u64, _u64, _u64, _vp, _vp])
_add = he._sig("he_ckks_add", _i32, [_vp, _vp, _vp, _u64, _vp, _vp])
_decrypt = he._sig("he_ckks_decrypt", _i32, [_vp, _vp, _u64, _vp, _vp])
_decode = he._sig("he_ckks_decode", _i32, [_vp, _vp, _u64, _u32, _vp, _vp])
_err = he._sig("he_ckks_last_error", ctypes.c_char_p, [])


def _check(rc: int) -> None:
    if rc != he.HE_OK:
        raise he.HEError(rc, (_err() or b"").decode())


class Context:
    """CKKS keys and tables on the current device."""

    def __init__(self, log_n: int = 14, scale_bits: int = 40, seed: int = 0):
        h = _vp()
        _check(_create(log_n, scale_bits, seed, ctypes.byref(h)))
        self._h = h
        n, sb = _u32(), _u32()
        primes = (_u32 * 3)()
        _check(_params(h, ctypes.byref(n), ctypes.cast(primes, _vp), ctypes.byref(sb)))
        self.n, self.scale_bits, self.primes = int(n.value), int(sb.value), [int(p) for p in primes]

    @property
    def slots(self) -> int:
        return self.n // 2

    def encode(self, z: torch.Tensor, stream=None) -> torch.Tensor:
        """z float64 [count, n_values] (n_values <= N/2) -> int32 [count, 3, N]."""
        assert z.dtype == torch.float64 and z.dim() == 2 and z.shape[1] <= self.slots
        z = z.contiguous()
        pt = torch.empty((z.shape[0], 3, self.n), dtype=torch.int32, device=z.device)
        _check(_encode(self._h, he._ptr(z), z.shape[0], z.shape[1], he._ptr(pt), he._stream(stream)))
        return pt

    def encrypt(self, pt: torch.Tensor, seed: int, offset: int = 0, out: Optional[torch.Tensor] = None,
                stream=None) -> torch.Tensor:
        assert pt.dtype == torch.int32 and pt.shape[1:] == (3, self.n)
        pt = pt.contiguous()
        if out is None:
            out = torch.empty((pt.shape[0], 2, 3, self.n), dtype=torch.int32, device=pt.device)
        _check(_encrypt(self._h, he._ptr(pt), pt.shape[0], seed, offset, he._ptr(out), he._stream(stream)))
        return out

    def add(self, x: torch.Tensor, y: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None):
        assert x.shape == y.shape and x.shape[1:] == (2, 3, self.n)
        x, y = x.contiguous(), y.contiguous()
        if out is None:
            out = torch.empty_like(x)
        _check(_add(self._h, he._ptr(x), he._ptr(y), x.shape[0], he._ptr(out), he._stream(stream)))
        return out

    def decrypt(self, ct: torch.Tensor, stream=None) -> torch.Tensor:
        assert ct.shape[1:] == (2, 3, self.n)
        ct = ct.contiguous()
        pt = torch.empty((ct.shape[0], 3, self.n), dtype=torch.int32, device=ct.device)
        _check(_decrypt(self._h, he._ptr(ct), ct.shape[0], he._ptr(pt), he._stream(stream)))
        return pt

    def decode(self, pt: torch.Tensor, n_values: int, stream=None) -> torch.Tensor:
        assert pt.shape[1:] == (3, self.n) and n_values <= self.slots
        pt = pt.contiguous()
        z = torch.empty((pt.shape[0], n_values), dtype=torch.float64, device=pt.device)
        _check(_decode(self._h, he._ptr(pt), pt.shape[0], n_values, he._ptr(z), he._stream(stream)))
        return z

    def close(self):
        if self._h and self._h.value:
            _free(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
