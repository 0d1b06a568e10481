"""Python binding of the gfx950 CKKS library (include/ckks.h).

Argument marshalling only: every step of every operation runs in the HIP
kernels of libckks.so.  PyTorch supplies device memory (uint64 tensors) and
streams; nothing here computes on the data.  If the library has not been built
the import fails: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libckks.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libckks.so is not built: run paper_2507_04775_amd/build.py (or __graft_entry__.build())")

_lib = ctypes.CDLL(LIB_PATH)

_vp = ctypes.c_void_p
_u32 = ctypes.c_uint32
_i32 = ctypes.c_int32
_u64p = ctypes.POINTER(ctypes.c_uint64)


class _Ct(ctypes.Structure):
    _fields_ = [("c0", _vp), ("c1", _vp), ("level", _u32), ("scale", ctypes.c_double)]


OP_MODUP, OP_MODDOWN, OP_KEYSWITCH, OP_HMULT, OP_RESCALE, OP_ROTATE, OP_HOISTED = 1, 2, 3, 4, 5, 6, 7
WORK_HMULT_RELIN, WORK_KEYSWITCH, WORK_ROTATE, WORK_HOISTED = 1, 2, 3, 4


class _Work(ctypes.Structure):
    _fields_ = [("kind", _u32), ("a", _Ct), ("b", _Ct), ("key", _vp), ("galois", _u32), ("n_rot", _u32),
                ("rot", ctypes.POINTER(_i32)), ("rot_keys", ctypes.POINTER(_vp)), ("out", ctypes.POINTER(_Ct))]

class _BootDesc(ctypes.Structure):
    _fields_ = [("n_cts", _u32), ("n_stc", _u32), ("cts_radix_logs", ctypes.POINTER(_u32)),
                ("stc_radix_logs", ctypes.POINTER(_u32)), ("cts_diags", ctypes.POINTER(_vp)),
                ("stc_diags", ctypes.POINTER(_vp)), ("cheb_degree", _u32), ("cheb", ctypes.POINTER(ctypes.c_double)),
                ("cheb_baby", _u32), ("double_angles", _u32), ("top_scale", ctypes.c_double), ("relin", _vp), ("conj", _vp),
                ("to_sparse", _vp), ("from_sparse", _vp),
                ("n_rot", _u32), ("rot_steps", ctypes.POINTER(_i32)), ("rot_keys", ctypes.POINTER(_vp)),
                ("hoist_moddown", _u32), ("input_gain", ctypes.c_uint64),
                ("device_buffer", _vp), ("device_buffer_bytes", ctypes.c_size_t)]


_sigs = {
    "ckks_ctx_create": (ctypes.c_int, [_u32, _u64p, _u32, _u64p, _u32, _u32, ctypes.c_int, ctypes.POINTER(_vp)]),
    "ckks_ctx_destroy": (None, [_vp]),
    "ckks_last_error": (ctypes.c_char_p, []),
    "ckks_sync": (ctypes.c_int, [_vp, _vp]),
    "ckks_workspace_bytes": (ctypes.c_size_t, [_vp, _u32, _u32]),
    "ckks_get_twiddles": (ctypes.c_int, [_vp, _u32, _u64p]),
    "ckks_ntt": (ctypes.c_int, [_vp, _vp, _u32, _u32, _vp]),
    "ckks_ntt_tile_set": (ctypes.c_int, [_u32, _u32, _u32]),
    "ckks_ntt_tile_get": (_u32, [_u32, _u32]),
    "ckks_intt": (ctypes.c_int, [_vp, _vp, _u32, _u32, _vp]),
    "ckks_modup": (ctypes.c_int, [_vp, _vp, _u32, _vp, _vp, _vp]),
    "ckks_inner_product": (ctypes.c_int, [_vp, _vp, _u32, _vp, _u32, _vp, _vp]),
    "ckks_moddown": (ctypes.c_int, [_vp, _vp, _u32, _vp, _vp, _vp]),
    "ckks_key_wrap": (ctypes.c_int, [_vp, _vp, _u32, ctypes.POINTER(_vp)]),
    "ckks_key_release": (None, [_vp]),
    "ckks_keyswitch": (ctypes.c_int, [_vp, _vp, _u32, _vp, _vp, _vp, _vp, _vp]),
    "ckks_keyswitch_noalloc": (ctypes.c_int, [_vp, _vp, _u32, _vp, _vp, _vp, _vp]),
    "ckks_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "ckks32_ctx_create": (ctypes.c_int, [_u32, ctypes.POINTER(_u32), _u32, ctypes.POINTER(_u32), _u32, _u32,
                                         ctypes.c_int, ctypes.POINTER(_vp)]),
    "ckks32_ctx_destroy": (None, [_vp]),
    "ckks32_workspace_bytes": (ctypes.c_size_t, [_vp, _u32, _u32]),
    "ckks32_ntt": (ctypes.c_int, [_vp, _vp, _u32, _u32, _vp]),
    "ckks32_intt": (ctypes.c_int, [_vp, _vp, _u32, _u32, _vp]),
    "ckks32_modup": (ctypes.c_int, [_vp, _vp, _u32, _vp, _vp, _vp]),
    "ckks32_moddown": (ctypes.c_int, [_vp, _vp, _u32, _vp, _vp, _vp, _vp]),
    "ckks32_keyswitch": (ctypes.c_int, [_vp, _vp, _u32, _vp, _vp, _vp, _vp, _vp]),
    "ckks32_hmult_relin": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _u32, _vp, _vp, _vp, _vp, _vp]),
    "ckks32_apply_galois": (ctypes.c_int, [_vp, _vp, _vp, _u32, _u32, _vp, _vp, _vp, _vp, _vp]),
    "ckks32_rescale": (ctypes.c_int, [_vp, _vp, _vp, _u32, _vp, _vp, _vp, _vp]),
    "ckks_probe_mad64": (ctypes.c_int, [_vp, _u32, _u32, _vp, ctypes.POINTER(ctypes.c_uint64)]),
    "ckks_hmult_relin": (ctypes.c_int, [_vp, ctypes.POINTER(_Ct), ctypes.POINTER(_Ct), _vp, ctypes.POINTER(_Ct), _vp, _vp]),
    "ckks_rescale": (ctypes.c_int, [_vp, ctypes.POINTER(_Ct), ctypes.POINTER(_Ct), _vp, _vp]),
    "ckks_apply_galois": (ctypes.c_int, [_vp, ctypes.POINTER(_Ct), _u32, _vp, ctypes.POINTER(_Ct), _vp, _vp]),
    "ckks_hrotate": (ctypes.c_int, [_vp, ctypes.POINTER(_Ct), _i32, _vp, ctypes.POINTER(_Ct), _vp, _vp]),
    "ckks_conjugate": (ctypes.c_int, [_vp, ctypes.POINTER(_Ct), _vp, ctypes.POINTER(_Ct), _vp, _vp]),
    "ckks_hrotate_hoisted": (ctypes.c_int, [_vp, ctypes.POINTER(_Ct), _u32, ctypes.POINTER(_i32), ctypes.POINTER(_vp),
                                            ctypes.POINTER(_Ct), _vp, _vp]),
    "ckks_poly_add": (ctypes.c_int, [_vp, _vp, _vp, _vp, _u32, _vp]),
    "ckks_poly_sub": (ctypes.c_int, [_vp, _vp, _vp, _vp, _u32, _vp]),
    "ckks_poly_mul": (ctypes.c_int, [_vp, _vp, _vp, _vp, _u32, _vp]),
    "ckks_poly_mul_add": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _u32, _vp]),
    "ckks_poly_scalar_mul": (ctypes.c_int, [_vp, _vp, _u64p, _vp, _u32, _vp]),
    "ckks_poly_scalar_add": (ctypes.c_int, [_vp, _vp, _u64p, _vp, _u32, _vp]),
    "ckks_automorph": (ctypes.c_int, [_vp, _vp, _u32, _vp, _u32, _vp]),
    "ckks_hadd": (ctypes.c_int, [_vp, ctypes.POINTER(_Ct), ctypes.POINTER(_Ct), ctypes.POINTER(_Ct), _vp]),
    "ckks_ptadd": (ctypes.c_int, [_vp, ctypes.POINTER(_Ct), _vp, ctypes.POINTER(_Ct), _vp]),
    "ckks_ptmult": (ctypes.c_int, [_vp, ctypes.POINTER(_Ct), _vp, ctypes.c_double, ctypes.POINTER(_Ct), _vp]),
    "ckks_scalar_add": (ctypes.c_int, [_vp, ctypes.POINTER(_Ct), _u64p, ctypes.POINTER(_Ct), _vp]),
    "ckks_scalar_mult": (ctypes.c_int, [_vp, ctypes.POINTER(_Ct), _u64p, ctypes.c_double, ctypes.POINTER(_Ct), _vp]),
    "ckks_hsquare": (ctypes.c_int, [_vp, ctypes.POINTER(_Ct), _vp, ctypes.POINTER(_Ct), _vp, _vp]),
    "ckks_batch_workspace_bytes": (ctypes.c_size_t, [_vp, ctypes.POINTER(_Work), _u32]),
    "ckks_batch_create": (ctypes.c_int, [_vp, ctypes.POINTER(_Work), _u32, _vp, ctypes.POINTER(_vp)]),
    "ckks_batch_run": (ctypes.c_int, [_vp, _vp]),
    "ckks_batch_tune": (ctypes.c_int, [_vp, _vp]),
    "ckks_batch_capture": (ctypes.c_int, [_vp, _vp]),
    "ckks_batch_replay": (ctypes.c_int, [_vp, _vp]),
    "ckks_batch_keyswitches": (_u32, [_vp]),
    "ckks_batch_grid": (_u32, [_vp, _u32]),
    "ckks_batch_set_grid": (ctypes.c_int, [_vp, _u32, _u32]),
    "ckks_batch_steps": (_u32, []),
    "ckks_batch_set_schedule": (ctypes.c_int, [_vp, _u32, _u32]),
    "ckks_batch_schedule": (_u32, [_vp]),
    "ckks_batch_faults": (ctypes.c_int, [_vp, _vp]),
    "ckks_batch_destroy": (None, [_vp]),
    "ckks_boot_create": (ctypes.c_int, [_vp, ctypes.POINTER(_BootDesc), ctypes.POINTER(_vp)]),
    "ckks_boot_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(_BootDesc), ctypes.POINTER(ctypes.c_size_t)]),
    "ckks_boot_output_level": (_u32, [_vp]),
    "ckks_boot_keyswitches": (_u32, [_vp]),
    "ckks_boot_device_bytes": (ctypes.c_size_t, [_vp]),
    "ckks_bootstrap": (ctypes.c_int, [_vp, ctypes.POINTER(_Ct), ctypes.POINTER(_Ct), _vp]),
    "ckks_boot_capture": (ctypes.c_int, [_vp, ctypes.POINTER(_Ct), ctypes.POINTER(_Ct), _vp]),
    "ckks_boot_replay": (ctypes.c_int, [_vp, _vp]),
    "ckks_boot_destroy": (None, [_vp]),
}
for _name, (_res, _args) in _sigs.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sigs)


def noalloc_scratch_bytes() -> int:
    """Size of the static scratch behind ckks_keyswitch_noalloc (bytes)."""
    return int(_lib.ckks_noalloc_scratch_bytes())


class CkksError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s failed with status %d: %s" % (where, status, _lib.ckks_last_error().decode()))


def _check(status: int, where: str):
    if status != 0:
        raise CkksError(status, where)


def _ptr32(t: Optional[torch.Tensor]):
    if t is None:
        return None
    assert t.dtype == torch.int32 and t.is_contiguous(), "expects contiguous tensors of 32-bit words (torch.int32)"
    return ctypes.c_void_p(t.data_ptr())


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    assert t.dtype == torch.uint64 and t.is_contiguous(), "expects contiguous uint64 tensors"
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _u64arr(xs):
    a = (ctypes.c_uint64 * len(xs))(*[int(x) for x in xs])
    return a


@dataclass
class Ciphertext:
    """Two device polynomials [level+1][N] (uint64) at `level`."""
    c0: torch.Tensor
    c1: torch.Tensor
    level: int
    scale: float = 1.0

    def _c(self) -> _Ct:
        return _Ct(_ptr(self.c0), _ptr(self.c1), self.level, self.scale)


class Key:
    """Device key [dnum][2][nq+np][N] wrapped for the library (kept alive here)."""

    def __init__(self, ctx: "Context", data: torch.Tensor, galois: int):
        self.ctx = ctx
        self.data = data
        self.galois = galois
        h = _vp()
        _check(_lib.ckks_key_wrap(ctx.handle, _ptr(data), galois, ctypes.byref(h)), "ckks_key_wrap")
        self.handle = h

    def __del__(self, _release=_lib.ckks_key_release):
        h = getattr(self, "handle", None)
        if h:
            _release(h)
            self.handle = None


class Context:
    """A parameter set [N, q_0..q_L, p_0..p_{K-1}, dnum] with its device tables."""

    def __init__(self, logn: int, q: Sequence[int], p: Sequence[int], dnum: int, device: int = 0):
        self.logn, self.N = int(logn), 1 << int(logn)
        self.q, self.p, self.dnum = [int(x) for x in q], [int(x) for x in p], int(dnum)
        self.nq, self.np = len(self.q), len(self.p)
        self.alpha = -(-self.nq // self.dnum)
        self.device = torch.device("cuda", device)
        h = _vp()
        _check(_lib.ckks_ctx_create(self.logn, _u64arr(self.q), self.nq, _u64arr(self.p), self.np, self.dnum,
                                    device, ctypes.byref(h)), "ckks_ctx_create")
        self.handle = h
        self._ws = {}

    def close(self, _destroy=_lib.ckks_ctx_destroy):
        if getattr(self, "handle", None):
            _destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()

    # ------------------------------------------------------------ helpers
    def beta(self, level: int) -> int:
        return -(-(level + 1) // self.alpha)

    def workspace_bytes(self, op: int, level: int) -> int:
        return int(_lib.ckks_workspace_bytes(self.handle, op, level))

    def workspace(self, op: int, level: int) -> torch.Tensor:
        """A cached device workspace large enough for `op` at `level`."""
        need = (self.workspace_bytes(op, level) + 7) // 8
        ws = self._ws.get(op)
        if ws is None or ws.numel() < need:
            ws = torch.empty(need, dtype=torch.uint64, device=self.device)
            self._ws[op] = ws
        return ws

    def empty_poly(self, level: int) -> torch.Tensor:
        return torch.empty((level + 1, self.N), dtype=torch.uint64, device=self.device)

    def empty_ct(self, level: int) -> Ciphertext:
        return Ciphertext(self.empty_poly(level), self.empty_poly(level), level)

    def key(self, data: torch.Tensor, galois: int) -> Key:
        return Key(self, data, galois)

    def sync(self, stream=None):
        _check(_lib.ckks_sync(self.handle, _stream(stream)), "ckks_sync")

    def twiddles(self, limb: int):
        import numpy as np
        out = np.zeros(self.N, dtype=np.uint64)
        _check(_lib.ckks_get_twiddles(self.handle, limb, out.ctypes.data_as(_u64p)), "ckks_get_twiddles")
        return out

    # ---------------------------------------------------------- the C ABI
    def ckks_ntt(self, poly: torch.Tensor, limb0: int = 0, n_limbs: Optional[int] = None, stream=None):
        n_limbs = poly.shape[0] if n_limbs is None else n_limbs
        _check(_lib.ckks_ntt(self.handle, _ptr(poly), limb0, n_limbs, _stream(stream)), "ckks_ntt")

    def ckks_intt(self, poly: torch.Tensor, limb0: int = 0, n_limbs: Optional[int] = None, stream=None):
        n_limbs = poly.shape[0] if n_limbs is None else n_limbs
        _check(_lib.ckks_intt(self.handle, _ptr(poly), limb0, n_limbs, _stream(stream)), "ckks_intt")

    def ckks_modup(self, d: torch.Tensor, level: int, ext: torch.Tensor, ws=None, stream=None):
        ws = self.workspace(OP_MODUP, level) if ws is None else ws
        _check(_lib.ckks_modup(self.handle, _ptr(d), level, _ptr(ext), _ptr(ws), _stream(stream)), "ckks_modup")

    def ckks_inner_product(self, ext: torch.Tensor, level: int, key: Key, galois: int, acc: torch.Tensor,
                           stream=None):
        _check(_lib.ckks_inner_product(self.handle, _ptr(ext), level, key.handle, galois, _ptr(acc),
                                       _stream(stream)), "ckks_inner_product")

    def ckks_moddown(self, x: torch.Tensor, level: int, out: torch.Tensor, ws=None, stream=None):
        ws = self.workspace(OP_MODDOWN, level) if ws is None else ws
        _check(_lib.ckks_moddown(self.handle, _ptr(x), level, _ptr(out), _ptr(ws), _stream(stream)), "ckks_moddown")

    def ckks_keyswitch(self, d: torch.Tensor, level: int, key: Key, out0: torch.Tensor, out1: torch.Tensor, ws=None,
                       stream=None):
        ws = self.workspace(OP_KEYSWITCH, level) if ws is None else ws
        _check(_lib.ckks_keyswitch(self.handle, _ptr(d), level, key.handle, _ptr(out0), _ptr(out1), _ptr(ws),
                                   _stream(stream)), "ckks_keyswitch")

    def ckks_keyswitch_noalloc(self, d: torch.Tensor, level: int, key: Key, out0: torch.Tensor, out1: torch.Tensor,
                               stream=None):
        _check(_lib.ckks_keyswitch_noalloc(self.handle, _ptr(d), level, key.handle, _ptr(out0), _ptr(out1),
                                           _stream(stream)), "ckks_keyswitch_noalloc")

    def ckks_hmult_relin(self, a: Ciphertext, b: Ciphertext, rlk: Key, out: Ciphertext, ws=None, stream=None):
        ws = self.workspace(OP_HMULT, a.level) if ws is None else ws
        ca, cb, co = a._c(), b._c(), out._c()
        _check(_lib.ckks_hmult_relin(self.handle, ctypes.byref(ca), ctypes.byref(cb), rlk.handle, ctypes.byref(co),
                                     _ptr(ws), _stream(stream)), "ckks_hmult_relin")
        out.level, out.scale = co.level, co.scale

    def ckks_hsquare(self, a: Ciphertext, rlk: Key, out: Ciphertext, ws=None, stream=None):
        ws = self.workspace(OP_HMULT, a.level) if ws is None else ws
        ca, co = a._c(), out._c()
        _check(_lib.ckks_hsquare(self.handle, ctypes.byref(ca), rlk.handle, ctypes.byref(co), _ptr(ws),
                                 _stream(stream)), "ckks_hsquare")
        out.level, out.scale = co.level, co.scale

    # Table I support operations on whole ciphertexts
    def ckks_hadd(self, a: Ciphertext, b: Ciphertext, out: Ciphertext, stream=None):
        ca, cb, co = a._c(), b._c(), out._c()
        _check(_lib.ckks_hadd(self.handle, ctypes.byref(ca), ctypes.byref(cb), ctypes.byref(co), _stream(stream)),
               "ckks_hadd")
        out.level, out.scale = co.level, co.scale

    def ckks_ptadd(self, a: Ciphertext, pt, out: Ciphertext, stream=None):
        ca, co = a._c(), out._c()
        _check(_lib.ckks_ptadd(self.handle, ctypes.byref(ca), _ptr(pt), ctypes.byref(co), _stream(stream)),
               "ckks_ptadd")
        out.level, out.scale = co.level, co.scale

    def ckks_ptmult(self, a: Ciphertext, pt, pt_scale: float, out: Ciphertext, stream=None):
        ca, co = a._c(), out._c()
        _check(_lib.ckks_ptmult(self.handle, ctypes.byref(ca), _ptr(pt), pt_scale, ctypes.byref(co),
                                _stream(stream)), "ckks_ptmult")
        out.level, out.scale = co.level, co.scale

    def ckks_scalar_add(self, a: Ciphertext, residues, out: Ciphertext, stream=None):
        ca, co = a._c(), out._c()
        _check(_lib.ckks_scalar_add(self.handle, ctypes.byref(ca), _u64arr(residues), ctypes.byref(co),
                                    _stream(stream)), "ckks_scalar_add")
        out.level, out.scale = co.level, co.scale

    def ckks_scalar_mult(self, a: Ciphertext, residues, scale: float, out: Ciphertext, stream=None):
        ca, co = a._c(), out._c()
        _check(_lib.ckks_scalar_mult(self.handle, ctypes.byref(ca), _u64arr(residues), scale, ctypes.byref(co),
                                     _stream(stream)), "ckks_scalar_mult")
        out.level, out.scale = co.level, co.scale

    def ckks_rescale(self, inp: Ciphertext, out: Ciphertext, ws=None, stream=None):
        ws = self.workspace(OP_RESCALE, inp.level) if ws is None else ws
        ci, co = inp._c(), out._c()
        _check(_lib.ckks_rescale(self.handle, ctypes.byref(ci), ctypes.byref(co), _ptr(ws), _stream(stream)),
               "ckks_rescale")
        out.level, out.scale = co.level, co.scale

    def ckks_apply_galois(self, inp: Ciphertext, galois: int, key: Key, out: Ciphertext, ws=None, stream=None):
        ws = self.workspace(OP_ROTATE, inp.level) if ws is None else ws
        ci, co = inp._c(), out._c()
        _check(_lib.ckks_apply_galois(self.handle, ctypes.byref(ci), galois, key.handle, ctypes.byref(co), _ptr(ws),
                                      _stream(stream)), "ckks_apply_galois")
        out.level, out.scale = co.level, co.scale

    def ckks_hrotate(self, inp: Ciphertext, k: int, key: Key, out: Ciphertext, ws=None, stream=None):
        ws = self.workspace(OP_ROTATE, inp.level) if ws is None else ws
        ci, co = inp._c(), out._c()
        _check(_lib.ckks_hrotate(self.handle, ctypes.byref(ci), k, key.handle, ctypes.byref(co), _ptr(ws),
                                 _stream(stream)), "ckks_hrotate")
        out.level, out.scale = co.level, co.scale

    def ckks_conjugate(self, inp: Ciphertext, key: Key, out: Ciphertext, ws=None, stream=None):
        ws = self.workspace(OP_ROTATE, inp.level) if ws is None else ws
        ci, co = inp._c(), out._c()
        _check(_lib.ckks_conjugate(self.handle, ctypes.byref(ci), key.handle, ctypes.byref(co), _ptr(ws),
                                   _stream(stream)), "ckks_conjugate")
        out.level, out.scale = co.level, co.scale

    def ckks_hrotate_hoisted(self, inp: Ciphertext, ks: Sequence[int], keys: Sequence[Key],
                             outs: Sequence[Ciphertext], ws=None, stream=None):
        n = len(ks)
        ws = self.workspace(OP_HOISTED, inp.level) if ws is None else ws
        ci = inp._c()
        karr = (_i32 * n)(*ks)
        harr = (_vp * n)(*[k.handle for k in keys])
        oarr = (_Ct * n)(*[o._c() for o in outs])
        _check(_lib.ckks_hrotate_hoisted(self.handle, ctypes.byref(ci), n, karr, harr, oarr, _ptr(ws),
                                         _stream(stream)), "ckks_hrotate_hoisted")
        for i, o in enumerate(outs):
            o.level, o.scale = oarr[i].level, oarr[i].scale

    def ckks_poly_add(self, a, b, out, level, stream=None):
        _check(_lib.ckks_poly_add(self.handle, _ptr(a), _ptr(b), _ptr(out), level, _stream(stream)), "ckks_poly_add")

    def ckks_poly_sub(self, a, b, out, level, stream=None):
        _check(_lib.ckks_poly_sub(self.handle, _ptr(a), _ptr(b), _ptr(out), level, _stream(stream)), "ckks_poly_sub")

    def ckks_poly_mul(self, a, b, out, level, stream=None):
        _check(_lib.ckks_poly_mul(self.handle, _ptr(a), _ptr(b), _ptr(out), level, _stream(stream)), "ckks_poly_mul")

    def ckks_poly_mul_add(self, a, b, c, out, level, stream=None):
        _check(_lib.ckks_poly_mul_add(self.handle, _ptr(a), _ptr(b), _ptr(c), _ptr(out), level, _stream(stream)),
               "ckks_poly_mul_add")

    def ckks_poly_scalar_mul(self, a, scalars, out, level, stream=None):
        _check(_lib.ckks_poly_scalar_mul(self.handle, _ptr(a), _u64arr(scalars), _ptr(out), level, _stream(stream)),
               "ckks_poly_scalar_mul")

    def ckks_poly_scalar_add(self, a, scalars, out, level, stream=None):
        _check(_lib.ckks_poly_scalar_add(self.handle, _ptr(a), _u64arr(scalars), _ptr(out), level, _stream(stream)),
               "ckks_poly_scalar_add")

    def ckks_automorph(self, inp, galois, out, n_limbs=None, stream=None):
        n_limbs = inp.shape[0] if n_limbs is None else n_limbs
        _check(_lib.ckks_automorph(self.handle, _ptr(inp), galois, _ptr(out), n_limbs, _stream(stream)),
               "ckks_automorph")


class Batch:
    """A batch of independent key-switching work items run by persistent
    work-queue kernels, one launch per step (ckks_batch_* in include/ckks.h).

    Add items with hmult/keyswitch/rotate/hoisted, then call build() once; the
    workspace is allocated here with torch and bound to the batch."""

    def __init__(self, ctx: "Context"):
        self.ctx = ctx
        self._items = []
        self._keep = []
        self.handle = None
        self.ws = None

    def hmult(self, a: Ciphertext, b: Ciphertext, rlk: Key, out: Ciphertext):
        out.level = a.level
        self._items.append((WORK_HMULT_RELIN, a, b, rlk, 0, None, None, [out]))

    def keyswitch(self, d: torch.Tensor, level: int, key: Key, out0: torch.Tensor, out1: torch.Tensor):
        a = Ciphertext(d, d, level)
        self._items.append((WORK_KEYSWITCH, a, None, key, 0, None, None, [Ciphertext(out0, out1, level)]))

    def rotate(self, a: Ciphertext, galois: int, key: Key, out: Ciphertext):
        out.level, out.scale = a.level, a.scale
        self._items.append((WORK_ROTATE, a, None, key, galois, None, None, [out]))

    def hoisted(self, a: Ciphertext, ks: Sequence[int], keys: Sequence[Key], outs: Sequence[Ciphertext]):
        for o in outs:
            o.level, o.scale = a.level, a.scale
        self._items.append((WORK_HOISTED, a, None, None, 0, list(ks), list(keys), list(outs)))

    def _works(self):
        n = len(self._items)
        arr = (_Work * n)()
        keep = []
        for i, (kind, a, b, key, g, ks, keys, outs) in enumerate(self._items):
            w = arr[i]
            w.kind = kind
            w.a = a._c()
            if b is not None:
                w.b = b._c()
            w.key = key.handle if key is not None else None
            w.galois = g
            outs_c = (_Ct * len(outs))(*[o._c() for o in outs])
            keep.append(outs_c)
            w.out = outs_c
            if kind == WORK_HOISTED:
                rot = (_i32 * len(ks))(*ks)
                rk = (_vp * len(keys))(*[k.handle for k in keys])
                keep += [rot, rk]
                w.n_rot = len(ks)
                w.rot = rot
                w.rot_keys = rk
        return arr, keep

    def build(self):
        arr, keep = self._works()
        nbytes = int(_lib.ckks_batch_workspace_bytes(self.ctx.handle, arr, len(self._items)))
        if nbytes == 0:
            raise CkksError(-1, "ckks_batch_workspace_bytes")
        self.ws = torch.empty((nbytes + 7) // 8, dtype=torch.uint64, device=self.ctx.device)
        h = _vp()
        _check(_lib.ckks_batch_create(self.ctx.handle, arr, len(self._items), self.ws.data_ptr(), ctypes.byref(h)),
               "ckks_batch_create")
        self.handle = h
        self._keep = keep
        return self

    @property
    def keyswitches(self) -> int:
        return int(_lib.ckks_batch_keyswitches(self.handle))

    def grid(self, step: int) -> int:
        return int(_lib.ckks_batch_grid(self.handle, step))

    def set_grid(self, step: int, wg_per_cu: int):
        _check(_lib.ckks_batch_set_grid(self.handle, step, wg_per_cu), "ckks_batch_set_grid")

    @staticmethod
    def steps() -> int:
        return int(_lib.ckks_batch_steps())

    def set_schedule(self, window: int, wg_per_cu: int = 2):
        """window 0: one persistent launch per step; window >= 1: the whole batch in one launch,
        items pipelined in windows of `window` (ckks_batch_set_schedule)."""
        _check(_lib.ckks_batch_set_schedule(self.handle, window, wg_per_cu), "ckks_batch_set_schedule")

    @property
    def schedule(self) -> int:
        return int(_lib.ckks_batch_schedule(self.handle))

    def faults(self, stream=None):
        _check(_lib.ckks_batch_faults(self.handle, _stream(stream)), "ckks_batch_faults")

    def run(self, stream=None):
        _check(_lib.ckks_batch_run(self.handle, _stream(stream)), "ckks_batch_run")

    def tune(self, stream=None):
        _check(_lib.ckks_batch_tune(self.handle, _stream(stream)), "ckks_batch_tune")

    def capture(self, stream):
        _check(_lib.ckks_batch_capture(self.handle, _stream(stream)), "ckks_batch_capture")

    def replay(self, stream=None):
        _check(_lib.ckks_batch_replay(self.handle, _stream(stream)), "ckks_batch_replay")

    def close(self, _destroy=_lib.ckks_batch_destroy):
        if getattr(self, "handle", None):
            _destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


class Boot:
    """A bootstrapping handle (ckks_boot_* in include/ckks.h): the schedule is
    derived by the library from the group sizes, the Chebyshev degree and the
    number of double-angle steps; the planned constants (plaintext diagonals as
    integer-valued float64 arrays [count][N], Chebyshev coefficients) and the
    keys are passed in."""

    def __init__(self, ctx: "Context", cts_radix_logs, stc_radix_logs, cts_diags, stc_diags, cheb,
                 double_angles: int, top_scale: float, relin: Key, conj: Key, rot_keys: dict, cheb_baby: int = 0,
                 sparse: Optional[tuple] = None, hoist_moddown: bool = False, input_gain: int = 1):
        import numpy as np
        self.ctx = ctx
        self._keys = [relin, conj] + list(rot_keys.values())
        # (to_sparse, from_sparse): switching keys s -> s' and s' -> s for sparse-secret encapsulation
        d = _BootDesc()
        d.n_cts, d.n_stc = len(cts_radix_logs), len(stc_radix_logs)
        cr = (_u32 * d.n_cts)(*cts_radix_logs)
        sr = (_u32 * d.n_stc)(*stc_radix_logs)
        arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in list(cts_diags) + list(stc_diags)]
        cd = (_vp * d.n_cts)(*[a.ctypes.data for a in arrs[: d.n_cts]])
        sd = (_vp * d.n_stc)(*[a.ctypes.data for a in arrs[d.n_cts:]])
        ch = np.ascontiguousarray(cheb, dtype=np.float64)
        steps = sorted(rot_keys)
        rs = (_i32 * max(1, len(steps)))(*steps)
        rk = (_vp * max(1, len(steps)))(*[rot_keys[k].handle for k in steps])
        d.cts_radix_logs, d.stc_radix_logs, d.cts_diags, d.stc_diags = cr, sr, cd, sd
        d.cheb_degree = len(ch) - 1
        d.cheb = ch.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.double_angles = double_angles
        d.cheb_baby = cheb_baby
        d.top_scale = top_scale
        d.relin, d.conj = relin.handle, conj.handle
        if sparse is not None:
            d.to_sparse, d.from_sparse = sparse[0].handle, sparse[1].handle
            self._keys += list(sparse)
        d.n_rot, d.rot_steps, d.rot_keys = len(steps), rs, rk
        d.hoist_moddown = 1 if hoist_moddown else 0
        d.input_gain = int(input_gain)
        # the handle's device memory is a torch allocation (ckks_boot_bytes, then device_buffer)
        nbytes = ctypes.c_size_t(0)
        _check(_lib.ckks_boot_bytes(ctx.handle, ctypes.byref(d), ctypes.byref(nbytes)), "ckks_boot_bytes")
        self._mem = torch.empty(((nbytes.value + 7) // 8,), dtype=torch.uint64, device=ctx.device)
        d.device_buffer, d.device_buffer_bytes = self._mem.data_ptr(), self._mem.numel() * 8
        h = _vp()
        _check(_lib.ckks_boot_create(ctx.handle, ctypes.byref(d), ctypes.byref(h)), "ckks_boot_create")
        self.handle = h
        self._captured = None

    @property
    def output_level(self) -> int:
        return int(_lib.ckks_boot_output_level(self.handle))

    @property
    def keyswitches(self) -> int:
        return int(_lib.ckks_boot_keyswitches(self.handle))

    @property
    def device_bytes(self) -> int:
        return int(_lib.ckks_boot_device_bytes(self.handle))

    def ckks_bootstrap(self, inp: Ciphertext, out: Ciphertext, stream=None):
        i, o = inp._c(), out._c()
        _check(_lib.ckks_bootstrap(self.handle, ctypes.byref(i), ctypes.byref(o), _stream(stream)), "ckks_bootstrap")
        out.level, out.scale = o.level, o.scale

    def capture(self, inp: Ciphertext, out: Ciphertext, stream):
        i, o = inp._c(), out._c()
        _check(_lib.ckks_boot_capture(self.handle, ctypes.byref(i), ctypes.byref(o), _stream(stream)),
               "ckks_boot_capture")
        out.level, out.scale = o.level, o.scale
        self._captured = (inp, out)

    def replay(self, stream=None):
        _check(_lib.ckks_boot_replay(self.handle, _stream(stream)), "ckks_boot_replay")

    def close(self, _destroy=_lib.ckks_boot_destroy):
        if getattr(self, "handle", None):
            _destroy(self.handle)
            self.handle = None
            if getattr(self, "_mem", None) is not None:
                # the handle's internal streams may still use the memory: wait before torch reuses it
                torch.cuda.synchronize(self._mem.device)
                self._mem = None

    def __del__(self):
        self.close()


class Context32:
    """A context of the 32-bit word path (ckks32_* in include/ckks.h): N = 2^16,
    every prime below 2^30.  Polynomials are [limbs][N] device tensors of
    32-bit words, held as torch.int32 (to_device32 / to_host32 reinterpret them
    as unsigned); keys are [dnum][2][n_q+n_p][N] such tensors."""

    def __init__(self, logn: int, q: Sequence[int], p: Sequence[int], dnum: int, device: int = 0):
        self.logn, self.N = logn, 1 << logn
        self.q, self.p, self.dnum = [int(x) for x in q], [int(x) for x in p], dnum
        self.nq, self.np = len(self.q), len(self.p)
        self.alpha = -(-self.nq // dnum)
        self.device = torch.device("cuda", device)
        qa = (_u32 * self.nq)(*self.q)
        pa = (_u32 * self.np)(*self.p)
        h = _vp()
        _check(_lib.ckks32_ctx_create(logn, qa, self.nq, pa, self.np, dnum, device, ctypes.byref(h)),
               "ckks32_ctx_create")
        self.handle = h

    def beta(self, level: int) -> int:
        return -(-(level + 1) // self.alpha)

    def workspace(self, op: int, level: int) -> torch.Tensor:
        need = int(_lib.ckks32_workspace_bytes(self.handle, op, level))
        return torch.empty((need + 15) // 16 * 4, dtype=torch.int32, device=self.device)

    def empty(self, *shape) -> torch.Tensor:
        return torch.empty(shape + (self.N,), dtype=torch.int32, device=self.device)

    def ntt(self, poly, limb0: int = 0, n_limbs: Optional[int] = None, stream=None):
        n = poly.shape[0] if n_limbs is None else n_limbs
        _check(_lib.ckks32_ntt(self.handle, _ptr32(poly), limb0, n, _stream(stream)), "ckks32_ntt")

    def intt(self, poly, limb0: int = 0, n_limbs: Optional[int] = None, stream=None):
        n = poly.shape[0] if n_limbs is None else n_limbs
        _check(_lib.ckks32_intt(self.handle, _ptr32(poly), limb0, n, _stream(stream)), "ckks32_intt")

    def modup(self, d, level: int, ext, ws=None, stream=None):
        ws = self.workspace(OP_KEYSWITCH, level) if ws is None else ws
        _check(_lib.ckks32_modup(self.handle, _ptr32(d), level, _ptr32(ext), _ptr32(ws), _stream(stream)), "ckks32_modup")

    def moddown(self, x, level: int, out0, out1, ws=None, stream=None):
        ws = self.workspace(OP_KEYSWITCH, level) if ws is None else ws
        _check(_lib.ckks32_moddown(self.handle, _ptr32(x), level, _ptr32(out0), _ptr32(out1), _ptr32(ws), _stream(stream)),
               "ckks32_moddown")

    def keyswitch(self, d, level: int, key, out0, out1, ws=None, stream=None):
        ws = self.workspace(OP_KEYSWITCH, level) if ws is None else ws
        _check(_lib.ckks32_keyswitch(self.handle, _ptr32(d), level, _ptr32(key), _ptr32(out0), _ptr32(out1), _ptr32(ws),
                                     _stream(stream)), "ckks32_keyswitch")

    def hmult_relin(self, a0, a1, b0, b1, level: int, rlk, out0, out1, ws=None, stream=None):
        ws = self.workspace(OP_HMULT, level) if ws is None else ws
        _check(_lib.ckks32_hmult_relin(self.handle, _ptr32(a0), _ptr32(a1), _ptr32(b0), _ptr32(b1), level, _ptr32(rlk),
                                       _ptr32(out0), _ptr32(out1), _ptr32(ws), _stream(stream)), "ckks32_hmult_relin")

    def apply_galois(self, c0, c1, level: int, galois: int, key, out0, out1, ws=None, stream=None):
        ws = self.workspace(OP_ROTATE, level) if ws is None else ws
        _check(_lib.ckks32_apply_galois(self.handle, _ptr32(c0), _ptr32(c1), level, galois, _ptr32(key), _ptr32(out0),
                                        _ptr32(out1), _ptr32(ws), _stream(stream)), "ckks32_apply_galois")

    def rescale(self, c0, c1, level: int, out0, out1, ws=None, stream=None):
        ws = self.workspace(OP_RESCALE, level) if ws is None else ws
        _check(_lib.ckks32_rescale(self.handle, _ptr32(c0), _ptr32(c1), level, _ptr32(out0), _ptr32(out1), _ptr32(ws),
                                   _stream(stream)), "ckks32_rescale")

    def close(self, _destroy=_lib.ckks32_ctx_destroy):
        if getattr(self, "handle", None):
            _destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


def to_device32(a, device="cuda") -> torch.Tensor:
    """numpy array of residues below 2^32 -> contiguous device tensor of 32-bit words (torch.int32)."""
    import numpy as np
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.uint64).astype(np.uint32)).view(np.int32)).to(device)


def to_host32(t: torch.Tensor):
    """Device tensor of 32-bit words -> numpy uint64 residues."""
    import numpy as np
    return t.cpu().numpy().view(np.uint32).astype(np.uint64)


def to_device(a, device="cuda") -> torch.Tensor:
    """numpy uint64 -> contiguous device tensor (plain copy)."""
    import numpy as np
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64)).to(device)


def to_host(t: torch.Tensor):
    return t.cpu().numpy()


def probe_mad64(out: torch.Tensor, blocks: int, iters: int, stream=None) -> int:
    """Launches the multiply-add rate probe (ckks_probe_mad64); returns the
    multiply-adds per lane the launch performs."""
    n = ctypes.c_uint64(0)
    _check(_lib.ckks_probe_mad64(_ptr(out), blocks, iters, _stream(stream), ctypes.byref(n)), "ckks_probe_mad64")
    return int(n.value)


def ntt_tile_set(inverse: bool, n_limbs: int, tile: int) -> None:
    """Tile width of the N = 2^16 NTT grid launches over n_limbs limbs (0: default)."""
    _check(_lib.ckks_ntt_tile_set(1 if inverse else 0, n_limbs, tile), "ckks_ntt_tile_set")


def ntt_tile_get(inverse: bool, n_limbs: int) -> int:
    return int(_lib.ckks_ntt_tile_get(1 if inverse else 0, n_limbs))
