"""ctypes binding of the u1mps C ABI (include/u1mps.h).

Argument marshalling only: every step of the gate path runs in the HIP
kernels of ``libu1mps.so``.  PyTorch supplies the device allocator (its
caching allocator) and the stream; nothing here computes on the state.

The library is loaded from this package's directory.  If it is missing the
import of this module fails loudly -- there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libu1mps.so")

MPS_OK = 0
STATUS_NAMES = {0: "MPS_OK", -1: "MPS_E_ARG", -2: "MPS_E_CHARGE", -3: "MPS_E_NOMEM",
                -4: "MPS_E_DEVICE", -5: "MPS_E_NOCONV", -6: "MPS_E_NUMERIC"}


class MPSError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class mps_z(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class mps_device(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("release", FREE_FN), ("ctx", C.c_void_p), ("stream", C.c_void_p)]


FORM_PLAIN_C128 = 0          # every step in complex128
FORM_SPLIT_BF16X3 = 1        # Theta's charge-triple products in split BF16 on the matrix cores


class mps_opts(C.Structure):
    _fields_ = [("chi_max", C.c_int), ("cutoff", C.c_double), ("zero_tol", C.c_double),
                ("max_sweeps", C.c_int), ("jacobi_tol", C.c_double), ("form", C.c_int),
                ("modulus", C.c_int), ("blocked_sweeps", C.c_int), ("select_scratch", C.c_int),
                ("sweep_graph", C.c_int), ("tile_tuning", C.c_int), ("jacobi_block", C.c_int),
                ("jacobi_lockstep", C.c_int)]


class mps_stats(C.Structure):
    _fields_ = [("gates", C.c_longlong), ("layers", C.c_longlong), ("sectors", C.c_longlong),
                ("sweeps", C.c_longlong), ("rotations", C.c_longlong),
                ("theta_flops", C.c_double), ("jacobi_flops", C.c_double), ("update_flops", C.c_double),
                ("theta_ms", C.c_double), ("jacobi_ms", C.c_double), ("jacobi_aux_ms", C.c_double),
                ("select_ms", C.c_double), ("update_ms", C.c_double),
                ("theta_launches", C.c_longlong), ("jacobi_launches", C.c_longlong),
                ("jacobi_aux_launches", C.c_longlong), ("select_launches", C.c_longlong),
                ("update_launches", C.c_longlong), ("polish_launches", C.c_longlong),
                ("max_discarded", C.c_double), ("min_margin", C.c_double),
                ("gemm_ms", C.c_double), ("gemm_launches", C.c_longlong),
                ("gemm_mfma_flops", C.c_double), ("split_ms", C.c_double), ("leak_total", C.c_double),
                ("graph_launches", C.c_longlong), ("host_plan_ms", C.c_double),
                ("tile_tunings", C.c_longlong), ("gemm_variant", C.c_int), ("jacobi_block", C.c_int),
                ("jacobi8_ms", C.c_double), ("jacobi8_flops", C.c_double), ("jacobi8_launches", C.c_longlong)]


EXPORTS = ["mps_default_opts", "mps_create", "mps_create_product", "mps_create_product_charges",
           "mps_charge_components", "mps_bond_charges", "mps_destroy", "mps_apply_gate",
           "mps_apply_layer", "mps_apply_layer_dense", "mps_apply_batch", "mps_truncate", "mps_amplitude", "mps_norm", "mps_norm_noalloc", "mps_sample", "mps_bond_sectors",
           "mps_bond_lambda", "mps_site_tensor", "mps_last_leaks", "mps_set_timing", "mps_get_stats",
           "mps_reset_stats", "mps_sync", "mps_last_error"]


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"u1mps HIP library not built: {path} is missing "
                          "(run __graft_entry__.build())")
    # PyTorch ships its own HIP runtime with the same SONAME as the system
    # one.  Loading torch first makes the library bind to that runtime, so the
    # streams and device memory torch hands over are valid in the library.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    P = C.POINTER
    h = C.c_void_p
    st = C.c_int
    sig = {
        "mps_default_opts": (None, [P(mps_opts)]),
        "mps_create": (st, [C.c_int, C.c_int, C.c_int, P(C.c_int), P(C.c_int), P(P(mps_z)),
                            P(P(C.c_double)), P(mps_opts), P(mps_device), P(h)]),
        "mps_create_product": (st, [C.c_int, C.c_int, P(C.c_int), P(mps_opts), P(mps_device), P(h)]),
        "mps_create_product_charges": (st, [C.c_int, C.c_int, P(C.c_int), C.c_int, P(C.c_int), P(mps_opts),
                                            P(mps_device), P(h)]),
        "mps_charge_components": (st, [h, P(C.c_int)]),
        "mps_bond_charges": (st, [h, C.c_int, C.c_int, P(C.c_int), P(C.c_int), P(C.c_int)]),
        "mps_destroy": (st, [h]),
        "mps_apply_gate": (st, [h, C.c_int, P(mps_z), P(C.c_double)]),
        "mps_apply_layer": (st, [h, C.c_int, P(C.c_int), P(mps_z), P(C.c_double)]),
        "mps_apply_layer_dense": (st, [h, C.c_int, P(C.c_int), P(mps_z), P(C.c_double)]),
        "mps_apply_batch": (st, [C.c_int, P(h), P(C.c_int), P(C.c_int), P(mps_z), P(C.c_double)]),
        "mps_truncate": (st, [h, C.c_int, C.c_int, C.c_double, P(C.c_double)]),
        "mps_amplitude": (st, [h, C.c_int, P(C.c_int), P(mps_z)]),
        "mps_norm": (st, [h, P(C.c_double)]),
        "mps_norm_noalloc": (st, [h, P(C.c_double)]),
        "mps_sample": (st, [h, C.c_int, P(C.c_double), P(C.c_int), P(C.c_double)]),
        "mps_bond_sectors": (st, [h, C.c_int, C.c_int, P(C.c_int), P(C.c_int), P(C.c_int)]),
        "mps_bond_lambda": (st, [h, C.c_int, C.c_int, P(C.c_int), P(C.c_double)]),
        "mps_site_tensor": (st, [h, C.c_int, C.c_size_t, P(C.c_int), P(C.c_int), P(mps_z)]),
        "mps_last_leaks": (st, [h, C.c_int, P(C.c_int), P(C.c_double)]),
        "mps_set_timing": (st, [h, C.c_int]),
        "mps_get_stats": (st, [h, P(mps_stats)]),
        "mps_reset_stats": (st, [h]),
        "mps_sync": (st, [h]),
        "mps_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def _check(status: int) -> None:
    if status != MPS_OK:
        raise MPSError(status, lib().mps_last_error().decode())


class TorchDevice:
    """Allocator and stream hooks backed by PyTorch's caching allocator."""

    def __init__(self, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible to PyTorch")
        self.torch = torch
        self.device = torch.cuda.current_device()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._live: Dict[int, int] = {}

        def _alloc(nbytes, _ctx):
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
                self._live[p] = nbytes
                return p
            except Exception:      # the library reports MPS_E_NOMEM
                return None

        delete = torch.cuda.caching_allocator_delete

        def _free(ptr, _ctx):
            # at interpreter shutdown the process returns device memory itself
            if ptr and not sys.is_finalizing():
                self._live.pop(ptr, None)
                delete(ptr)

        self._alloc_cb = ALLOC_FN(_alloc)
        self._free_cb = FREE_FN(_free)

    def struct(self) -> mps_device:
        d = mps_device()
        d.alloc = self._alloc_cb
        d.release = self._free_cb
        d.ctx = None
        d.stream = C.c_void_p(self.stream.cuda_stream)
        return d


_OPEN: "weakref.WeakSet[MPS]" = weakref.WeakSet()


@atexit.register
def _close_all() -> None:
    # release handles while torch (their allocator) is still alive
    for m in list(_OPEN):
        try:
            m.close()
        except Exception:
            pass


class MPS:
    """A U(1)-symmetric MPS on the GPU, created as a Fock product state.
    modulus n >= 2 (with d <= n) makes the charge the particle number mod n;
    charge_map (d x K integers, K = 1 or 2) gives every local state its own
    charge with K independent U(1) components (mps_create_product_charges)."""

    def __init__(self, occupation: Sequence[int], d: int, chi_max: int = 0, cutoff: float = 0.0,
                 zero_tol: float = 1e-13, max_sweeps: int = 40, jacobi_tol: float = 0.0,
                 device: Optional[TorchDevice] = None, form: int = FORM_PLAIN_C128, modulus: int = 0,
                 blocked_sweeps: int = 0, select_scratch: int = 0, sweep_graph: int = 0, charge_map=None,
                 tile_tuning: int = 1, jacobi_block: int = 0, jacobi_lockstep: int = 0, _handle=None):
        self._lib = lib()
        self.L = len(occupation)
        self.d = d
        self.N = int(sum(occupation))
        self.modulus = int(modulus)
        self.ncomp = 1
        self._cap = max(self.N + 1, self.modulus)
        self._dev = device if device is not None else TorchDevice()
        self._dev_struct = self._dev.struct()
        self._opts = mps_opts(chi_max, cutoff, zero_tol, max_sweeps, jacobi_tol, int(form), int(modulus),
                              int(blocked_sweeps), int(select_scratch), int(sweep_graph), int(tile_tuning),
                              int(jacobi_block), int(jacobi_lockstep))
        self._h = C.c_void_p()
        if _handle is not None:
            self._h = _handle
            return
        occ = (C.c_int * self.L)(*[int(x) for x in occupation])
        if charge_map is None:
            _check(self._lib.mps_create_product(self.L, d, occ, C.byref(self._opts),
                                                C.byref(self._dev_struct), C.byref(self._h)))
        else:
            cm = np.asarray(charge_map, dtype=np.int64).reshape(d, -1)
            self.ncomp = int(cm.shape[1])
            flat = (C.c_int * cm.size)(*[int(x) for x in cm.reshape(-1)])
            _check(self._lib.mps_create_product_charges(self.L, d, occ, self.ncomp, flat, C.byref(self._opts),
                                                        C.byref(self._dev_struct), C.byref(self._h)))
            # sectors per bond: at most the number of distinct component tuples
            tot = cm[[int(x) for x in occupation]].sum(axis=0)
            self._cap = int(np.prod(tot + 1))
            self.total = tuple(int(x) for x in tot)
        _OPEN.add(self)

    @classmethod
    def from_vidal(cls, d: int, n_photons: int, bond_charges: List[Sequence[int]],
                   gammas: List[np.ndarray], lambdas: List[np.ndarray], chi_max: int = 0,
                   cutoff: float = 0.0, zero_tol: float = 1e-13, max_sweeps: int = 40,
                   jacobi_tol: float = 0.0, device: Optional[TorchDevice] = None,
                   form: int = FORM_PLAIN_C128, modulus: int = 0, blocked_sweeps: int = 0,
                   select_scratch: int = 0, sweep_graph: int = 0, tile_tuning: int = 1,
                   jacobi_block: int = 0, jacobi_lockstep: int = 0) -> "MPS":
        L = len(gammas)
        dims = [len(c) for c in bond_charges]
        obj = cls.__new__(cls)
        obj._lib = lib()
        obj.L, obj.d, obj.N = L, d, n_photons
        obj.modulus = int(modulus)
        obj.ncomp = 1
        obj._cap = max(n_photons + 1, obj.modulus)
        obj._dev = device if device is not None else TorchDevice()
        obj._dev_struct = obj._dev.struct()
        obj._opts = mps_opts(chi_max, cutoff, zero_tol, max_sweeps, jacobi_tol, int(form), int(modulus),
                             int(blocked_sweeps), int(select_scratch), int(sweep_graph), int(tile_tuning),
                             int(jacobi_block), int(jacobi_lockstep))
        obj._h = C.c_void_p()
        c_dims = (C.c_int * (L + 1))(*dims)
        flat = [int(c) for b in bond_charges for c in b]
        c_ch = (C.c_int * len(flat))(*flat)
        g_keep = [np.ascontiguousarray(np.asarray(g, dtype=np.complex128)) for g in gammas]
        l_keep = [np.ascontiguousarray(np.asarray(l, dtype=np.float64)) for l in lambdas]
        g_ptrs = (C.POINTER(mps_z) * L)(*[g.ctypes.data_as(C.POINTER(mps_z)) for g in g_keep])
        l_ptrs = (C.POINTER(C.c_double) * (L + 1))(*[l.ctypes.data_as(C.POINTER(C.c_double)) for l in l_keep])
        _check(obj._lib.mps_create(L, d, n_photons, c_dims, c_ch, g_ptrs, l_ptrs, C.byref(obj._opts),
                                   C.byref(obj._dev_struct), C.byref(obj._h)))
        _OPEN.add(obj)
        return obj

    # -------------------------------------------------------------- lifetime
    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            self._lib.mps_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # --------------------------------------------------------------- updates
    def apply_gate(self, site: int, u: np.ndarray) -> float:
        disc = C.c_double(0.0)
        zu = np.ascontiguousarray(np.asarray(u, dtype=np.complex128).reshape(2, 2))
        _check(self._lib.mps_apply_gate(self._h, int(site), zu.ctypes.data_as(C.POINTER(mps_z)),
                                        C.byref(disc)))
        return disc.value

    def apply_layer(self, sites: Sequence[int], us: Sequence[np.ndarray]) -> np.ndarray:
        n = len(sites)
        disc = np.zeros(n, dtype=np.float64)
        if n == 0:
            return disc
        c_sites = (C.c_int * n)(*[int(s) for s in sites])
        zu = np.ascontiguousarray(np.stack([np.asarray(u, dtype=np.complex128).reshape(2, 2) for u in us]))
        _check(self._lib.mps_apply_layer(self._h, n, c_sites, zu.ctypes.data_as(C.POINTER(mps_z)),
                                         disc.ctypes.data_as(C.POINTER(C.c_double))))
        return disc

    def apply_layer_dense(self, sites: Sequence[int], g4s: Sequence[np.ndarray]) -> np.ndarray:
        """Dense two-site gates, each d^2 x d^2 with row p*d+q and column a*d+b."""
        n = len(sites)
        disc = np.zeros(n, dtype=np.float64)
        if n == 0:
            return disc
        dd = self.d * self.d
        c_sites = (C.c_int * n)(*[int(s) for s in sites])
        zg = np.ascontiguousarray(np.stack([np.asarray(g, dtype=np.complex128).reshape(dd, dd) for g in g4s]))
        _check(self._lib.mps_apply_layer_dense(self._h, n, c_sites, zg.ctypes.data_as(C.POINTER(mps_z)),
                                               disc.ctypes.data_as(C.POINTER(C.c_double))))
        return disc

    def truncate(self, bond: int, chi_max: int, cutoff: float) -> float:
        disc = C.c_double(0.0)
        _check(self._lib.mps_truncate(self._h, int(bond), int(chi_max), float(cutoff), C.byref(disc)))
        return disc.value

    # ------------------------------------------------------------- read-outs
    def amplitudes(self, patterns) -> np.ndarray:
        pats = np.ascontiguousarray(np.asarray(patterns, dtype=np.int32).reshape(-1, self.L))
        out = np.zeros(pats.shape[0], dtype=np.complex128)
        if pats.shape[0]:
            _check(self._lib.mps_amplitude(self._h, pats.shape[0], pats.ctypes.data_as(C.POINTER(C.c_int)),
                                           out.ctypes.data_as(C.POINTER(mps_z))))
        return out

    def norm2(self) -> float:
        v = C.c_double(0.0)
        _check(self._lib.mps_norm(self._h, C.byref(v)))
        return v.value

    def norm2_noalloc(self) -> float:
        """<psi|psi> through mps_norm_noalloc (no device allocation)."""
        v = C.c_double(0.0)
        _check(self._lib.mps_norm_noalloc(self._h, C.byref(v)))
        return v.value

    def sample(self, uniforms: np.ndarray):
        """Exact samples: uniforms [count, L] in [0, 1) -> (patterns [count, L]
        int32, probabilities [count])."""
        u = np.ascontiguousarray(np.asarray(uniforms, dtype=np.float64).reshape(-1, self.L))
        n = u.shape[0]
        occ = np.zeros((n, self.L), dtype=np.int32)
        prob = np.zeros(n, dtype=np.float64)
        if n:
            _check(self._lib.mps_sample(self._h, n, u.ctypes.data_as(C.POINTER(C.c_double)),
                                        occ.ctypes.data_as(C.POINTER(C.c_int)),
                                        prob.ctypes.data_as(C.POINTER(C.c_double))))
        return occ, prob

    def bond_sectors(self, bond: int) -> Dict:
        """Charge -> multiplicity of a bond; with a two-component charge map the
        charges are (c1, c2) tuples."""
        cap = self._cap
        n = C.c_int(0)
        cnt = (C.c_int * cap)()
        if self.ncomp == 2:
            ch = (C.c_int * (2 * cap))()
            _check(self._lib.mps_bond_charges(self._h, int(bond), cap, C.byref(n), ch, cnt))
            return {(int(ch[2 * i]), int(ch[2 * i + 1])): int(cnt[i]) for i in range(n.value)}
        ch = (C.c_int * cap)()
        _check(self._lib.mps_bond_sectors(self._h, int(bond), cap, C.byref(n), ch, cnt))
        return {int(ch[i]): int(cnt[i]) for i in range(n.value)}

    def bond_dims(self) -> List[int]:
        return [sum(self.bond_sectors(b).values()) for b in range(self.L + 1)]

    def bond_lambda(self, bond: int) -> np.ndarray:
        dim = sum(self.bond_sectors(bond).values())
        out = np.zeros(dim, dtype=np.float64)
        n = C.c_int(0)
        _check(self._lib.mps_bond_lambda(self._h, int(bond), dim, C.byref(n),
                                         out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def site_tensor(self, site: int) -> np.ndarray:
        r = sum(self.bond_sectors(site).values())
        c = sum(self.bond_sectors(site + 1).values())
        out = np.zeros((r, c), dtype=np.complex128)
        rr, cc = C.c_int(0), C.c_int(0)
        _check(self._lib.mps_site_tensor(self._h, int(site), out.size, C.byref(rr), C.byref(cc),
                                         out.ctypes.data_as(C.POINTER(mps_z))))
        return out

    def last_leaks(self) -> np.ndarray:
        """Per-gate weight removed by the local cutoff in the last apply call."""
        n = C.c_int(0)
        self._lib.mps_last_leaks(self._h, 0, C.byref(n), None)
        out = np.zeros(max(n.value, 1), dtype=np.float64)
        _check(self._lib.mps_last_leaks(self._h, out.size, C.byref(n), out.ctypes.data_as(C.POINTER(C.c_double))))
        return out[:n.value]

    def set_timing(self, on: bool) -> None:
        _check(self._lib.mps_set_timing(self._h, 1 if on else 0))

    def stats(self) -> Dict[str, float]:
        s = mps_stats()
        _check(self._lib.mps_get_stats(self._h, C.byref(s)))
        out = {}
        for name, _ in mps_stats._fields_:
            v = getattr(s, name)
            out[name] = list(v) if isinstance(v, C.Array) else v
        return out

    def reset_stats(self) -> None:
        _check(self._lib.mps_reset_stats(self._h))

    def sync(self) -> None:
        _check(self._lib.mps_sync(self._h))


def apply_batch(states: Sequence["MPS"], layers: Sequence[Tuple[Sequence[int], Sequence[np.ndarray]]]
                ) -> List[np.ndarray]:
    """One layer of each state in one call of mps_apply_batch (the batching form).

    layers[i] = (sites, us) for states[i]; empty layers are allowed.  Returns
    each state's discarded weights."""
    if len(states) != len(layers):
        raise ValueError("one layer per state")
    n = len(states)
    if n == 0:
        return []
    lib_ = states[0]._lib
    hs = (C.c_void_p * n)(*[m._h for m in states])
    counts = [len(s) for s, _ in layers]
    total = sum(counts)
    c_counts = (C.c_int * n)(*counts)
    c_sites = (C.c_int * max(total, 1))(*[int(x) for s, _ in layers for x in s])
    mats = [np.asarray(u, dtype=np.complex128).reshape(2, 2) for _, us in layers for u in us]
    if len(mats) != total:
        raise ValueError("one 2x2 matrix per gate")
    zu = np.ascontiguousarray(np.stack(mats)) if mats else np.zeros((1, 2, 2), dtype=np.complex128)
    disc = np.zeros(max(total, 1), dtype=np.float64)
    _check(lib_.mps_apply_batch(n, hs, c_counts, c_sites, zu.ctypes.data_as(C.POINTER(mps_z)),
                                disc.ctypes.data_as(C.POINTER(C.c_double))))
    out, o = [], 0
    for c in counts:
        out.append(disc[o:o + c].copy())
        o += c
    return out
