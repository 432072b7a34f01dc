"""Python binding of the tdmps C ABI (ctypes; argument marshalling only).

Every operation runs in the HIP library `libtdmps.so` built in this package directory;
importing this module does not compute anything.  The names follow include/tdmps.h.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_LIB = os.path.join(_HERE, "libtdmps.so")

FP64, FP32, BF16X3, BF16X6 = 0, 1, 2, 3
KRYLOV_ORTHO, KRYLOV_NONORTHO = 0, 1

STATUS = {0: "OK", -1: "ERR_ARG", -2: "ERR_SECTOR", -3: "ERR_OOM", -4: "ERR_HIP", -5: "ERR_NUMERIC",
          -6: "ERR_SINGULAR", -7: "ERR_UNSUPPORTED"}


class TdmpsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class FitParams(ct.Structure):
    _fields_ = [("Dmax", ct.c_int32), ("n_sweeps", ct.c_int32), ("conv_tol", ct.c_double),
                ("svd_cutoff", ct.c_double), ("precision", ct.c_int32), ("batched", ct.c_int32)]


class FitInfo(ct.Structure):
    _fields_ = [("sweeps_used", ct.c_int32), ("max_bond", ct.c_int32), ("discarded_max", ct.c_double),
                ("discarded_sum", ct.c_double), ("norm2", ct.c_double)]


class Pulse(ct.Structure):
    """E(t) = amplitude * sin(omega t) * exp(-(t - t_center)^2 / (2 width^2))."""
    _fields_ = [("amplitude", ct.c_double), ("omega", ct.c_double), ("t_center", ct.c_double),
                ("width", ct.c_double)]


def fit_params(Dmax=64, n_sweeps=2, conv_tol=0.0, svd_cutoff=1e-12, precision=FP64, batched=1):
    return FitParams(Dmax, n_sweeps, conv_tol, svd_cutoff, precision, batched)


_P = ct.c_void_p
_PP = ct.POINTER(ct.c_void_p)
_D = ct.POINTER(ct.c_double)
_I32 = ct.POINTER(ct.c_int32)
_I64 = ct.POINTER(ct.c_int64)
_U8 = ct.POINTER(ct.c_uint8)

NCOUNTERS = 21  # TDMPS_NCOUNTERS of include/tdmps.h
TILE_CONFIGS = 10  # TDMPS_TILE_CONFIGS
TILE_BUCKETS = 192  # TDMPS_TILE_BUCKETS

_SIGS = {
    "tdmps_last_error": (ct.c_char_p, []),
    "tdmps_ctx_create": (ct.c_int32, [ct.c_int32, _P, _PP]),
    "tdmps_ctx_destroy": (ct.c_int32, [_P]),
    "tdmps_ctx_counters": (ct.c_int32, [_P, _D]),
    "tdmps_ctx_reset_counters": (ct.c_int32, [_P]),
    "tdmps_ctx_set_launch_mode": (ct.c_int32, [_P, ct.c_int32]),
    "tdmps_ctx_set_tile_config": (ct.c_int32, [_P, ct.c_int32]),
    "tdmps_ctx_autotune": (ct.c_int32, [_P, ct.c_int32, _I32, _D]),
    "tdmps_ctx_clear_tuning": (ct.c_int32, [_P]),
    "tdmps_mpo_from_integrals": (ct.c_int32, [_P, ct.c_int32, _D, _D, ct.c_double, _PP]),
    "tdmps_fiedler_order": (ct.c_int32, [ct.c_int32, _D, ct.c_void_p, _I32]),
    "tdmps_mpo_one_body": (ct.c_int32, [_P, ct.c_int32, _D, _PP]),
    "tdmps_mpo_set_one_body": (ct.c_int32, [_P, _D]),
    "tdmps_mpo_bond_dims": (ct.c_int32, [_P, _I32]),
    "tdmps_mpo_to_dense": (ct.c_int32, [_P, _D, ct.c_int64]),
    "tdmps_mpo_det_element": (ct.c_int32, [_P, _U8, _U8, _D]),
    "tdmps_mpo_destroy": (ct.c_int32, [_P]),
    "tdmps_mps_from_determinant": (ct.c_int32, [_P, ct.c_int32, _U8, _PP]),
    "tdmps_mps_from_blocks": (ct.c_int32, [_P, ct.c_int32, _I32, _I32, _D, ct.c_int64, _PP]),
    "tdmps_mps_sectors": (ct.c_int32, [_P, _I32, _I32, _I64]),
    "tdmps_mps_get_blocks": (ct.c_int32, [_P, _D, _I64]),
    "tdmps_mps_to_dense": (ct.c_int32, [_P, _D, ct.c_int64]),
    "tdmps_mps_from_dense": (ct.c_int32, [_P, ct.c_int32, ct.c_int32, ct.c_int32, _D, ct.c_int64, ct.c_int32,
                                          ct.c_double, _PP]),
    "tdmps_mps_save": (ct.c_int32, [_P, ct.c_char_p]),
    "tdmps_mps_load": (ct.c_int32, [_P, ct.c_char_p, _PP]),
    "tdmps_mps_copy": (ct.c_int32, [_P, _PP]),
    "tdmps_mps_bond_dims": (ct.c_int32, [_P, _I32]),
    "tdmps_mps_destroy": (ct.c_int32, [_P]),
    "tdmps_mps_scale": (ct.c_int32, [_P, _D]),
    "tdmps_mps_overlap": (ct.c_int32, [_P, _P, _D]),
    "tdmps_mps_expect": (ct.c_int32, [_P, _P, _P, _D]),
    "tdmps_mps_apply_H": (ct.c_int32, [_P, _D, _P, ct.c_int32, _D, _PP, ct.POINTER(FitParams), _PP,
                                       ct.POINTER(FitInfo)]),
    "tdmps_mps_compress": (ct.c_int32, [ct.c_int32, _D, _PP, ct.POINTER(FitParams), _PP, ct.POINTER(FitInfo)]),
    "tdmps_mps_annihilate": (ct.c_int32, [_P, ct.c_int32, ct.c_int32, _PP]),
    "tdmps_krylov_ground": (ct.c_int32, [_P, _P, ct.c_int32, ct.c_int32, ct.POINTER(FitParams), _PP, _D]),
    "tdmps_mps_one_rdm": (ct.c_int32, [_P, _D]),
    "tdmps_krylov_step": (ct.c_int32, [_P, _P, ct.c_double, ct.c_int32, ct.c_int32, ct.POINTER(FitParams), _PP,
                                       _D, _D]),
    "tdmps_rk4_step": (ct.c_int32, [_P, _P, _P, _P, ct.c_double, ct.POINTER(FitParams), _PP,
                                    ct.POINTER(FitInfo)]),
    "tdmps_heff_create": (ct.c_int32, [_P, _P, _P, ct.c_int32, ct.c_int32, _PP]),
    "tdmps_heff_layout": (ct.c_int32, [_P, ct.c_int32, _I64, _I64, _I32]),
    "tdmps_heff_apply": (ct.c_int32, [_P, _P, _P]),
    "tdmps_heff_apply_noalloc": (ct.c_int32, [_P, _P, _P]),
    "tdmps_heff_set_precision": (ct.c_int32, [_P, ct.c_int32]),
    "tdmps_heff_flops": (ct.c_int32, [_P, _D]),
    "tdmps_heff_destroy": (ct.c_int32, [_P]),
    "tdmps_pulse_forward": (ct.c_int32, [_P, _D, _D, _P, _P, ct.POINTER(Pulse), ct.c_double, ct.c_int32, ct.c_int32,
                                         ct.POINTER(FitParams), _PP, _D]),
    "tdmps_pulse_backward": (ct.c_int32, [_P, _D]),
    "tdmps_traj_destroy": (ct.c_int32, [_P]),
}

_LIB = None


def load(path: str | None = None):
    """Load the library (default: the in-tree build).  Fails loudly if it is missing."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or DEFAULT_LIB
    if not os.path.exists(p):
        raise RuntimeError(f"tdmps library not built: {p} (run __graft_entry__.build())")
    lib = ct.CDLL(p)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _LIB = lib
    return lib


def symbols():
    return list(_SIGS)


def _check(code):
    if code != 0:
        raise TdmpsError(code, _LIB.tdmps_last_error().decode())


def _dp(a):
    return a.ctypes.data_as(_D)


def _cplx(z):
    z = complex(z)
    return np.array([z.real, z.imag], dtype=np.float64)


class Context:
    def __init__(self, device=0, stream=None):
        load()
        h = ct.c_void_p()
        _check(_LIB.tdmps_ctx_create(device, ct.c_void_p(stream) if stream else None, ct.byref(h)))
        self.h = h

    def counters(self):
        out = np.zeros(NCOUNTERS)
        _check(_LIB.tdmps_ctx_counters(self.h, _dp(out)))
        return out

    def reset_counters(self):
        _check(_LIB.tdmps_ctx_reset_counters(self.h))

    def set_launch_mode(self, batched):
        """1: grouped launch per contraction stage (default); 2: grouped launches replayed from a
        captured HIP graph; 0: one launch per block product."""
        _check(_LIB.tdmps_ctx_set_launch_mode(self.h, int(batched)))

    def set_tile_config(self, cfg):
        """Force one grouped-GEMM tile shape (0..TILE_CONFIGS-1); -1 restores the automatic choice."""
        _check(_LIB.tdmps_ctx_set_tile_config(self.h, int(cfg)))

    def autotune(self, precision=FP64):
        """Times every tile shape per block-size bucket; returns (cfg, tflops) arrays of shape
        (8, 8, 3) over (row bucket, column bucket, reduction bucket)."""
        cfg = np.zeros(TILE_BUCKETS, dtype=np.int32)
        tf = np.zeros(TILE_BUCKETS)
        _check(_LIB.tdmps_ctx_autotune(self.h, int(precision), cfg.ctypes.data_as(_I32), _dp(tf)))
        return cfg.reshape(8, 8, 3), tf.reshape(8, 8, 3)

    def clear_tuning(self):
        _check(_LIB.tdmps_ctx_clear_tuning(self.h))

    def close(self):
        if self.h:
            _check(_LIB.tdmps_ctx_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MPO:
    def __init__(self, handle, L):
        self.h, self.L = handle, L

    @classmethod
    def from_integrals(cls, ctx, h, eri, e0=0.0):
        load()
        L = h.shape[0]
        h = np.ascontiguousarray(h, dtype=np.float64)
        eri = np.ascontiguousarray(eri, dtype=np.float64)
        out = ct.c_void_p()
        _check(_LIB.tdmps_mpo_from_integrals(ctx.h if ctx else None, L, _dp(h), _dp(eri), float(e0), ct.byref(out)))
        return cls(out, L)

    @classmethod
    def one_body(cls, ctx, t):
        load()
        t = np.ascontiguousarray(t, dtype=np.float64)
        out = ct.c_void_p()
        _check(_LIB.tdmps_mpo_one_body(ctx.h if ctx else None, t.shape[0], _dp(t), ct.byref(out)))
        return cls(out, t.shape[0])

    def set_one_body(self, h):
        h = np.ascontiguousarray(h, dtype=np.float64)
        _check(_LIB.tdmps_mpo_set_one_body(self.h, _dp(h)))

    def bond_dims(self):
        out = np.zeros(self.L + 1, dtype=np.int32)
        _check(_LIB.tdmps_mpo_bond_dims(self.h, out.ctypes.data_as(_I32)))
        return out

    def to_dense(self):
        n = 4 ** self.L
        out = np.zeros(n * n)
        _check(_LIB.tdmps_mpo_to_dense(self.h, _dp(out), n * n))
        return out.reshape(n, n)

    def det_element(self, bra, ket):
        b = np.ascontiguousarray(bra, dtype=np.uint8)
        k = np.ascontiguousarray(ket, dtype=np.uint8)
        out = ct.c_double()
        _check(_LIB.tdmps_mpo_det_element(self.h, b.ctypes.data_as(_U8), k.ctypes.data_as(_U8), ct.byref(out)))
        return out.value

    def close(self):
        if self.h:
            _check(_LIB.tdmps_mpo_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MPS:
    def __init__(self, handle, L):
        self.h, self.L = handle, L

    @classmethod
    def from_determinant(cls, ctx, occ):
        occ = np.ascontiguousarray(occ, dtype=np.uint8)
        out = ct.c_void_p()
        _check(_LIB.tdmps_mps_from_determinant(ctx.h, len(occ), occ.ctypes.data_as(_U8), ct.byref(out)))
        return cls(out, len(occ))

    @classmethod
    def from_blocks(cls, ctx, bonds, data):
        """bonds: list of L+1 lists of (n_up, n_dn, dim) ascending; data: complex site tensors
        concatenated in the panel layout."""
        L = len(bonds) - 1
        nsec = np.array([len(b) for b in bonds], dtype=np.int32)
        sec = np.array([x for b in bonds for s in b for x in s], dtype=np.int32)
        d = np.ascontiguousarray(np.asarray(data, dtype=np.complex128)).view(np.float64)
        out = ct.c_void_p()
        _check(_LIB.tdmps_mps_from_blocks(ctx.h, L, nsec.ctypes.data_as(_I32), sec.ctypes.data_as(_I32), _dp(d),
                                          d.size, ct.byref(out)))
        return cls(out, L)

    @classmethod
    def from_dense(cls, ctx, vec, n_up, n_dn, Dmax=1 << 30, svd_cutoff=1e-12):
        """Sequential-SVD state of a dense 4^L vector (zero outside the (n_up, n_dn) sector)."""
        v = np.ascontiguousarray(np.asarray(vec, dtype=np.complex128)).view(np.float64)
        L = int(round(np.log(v.size // 2) / np.log(4)))
        out = ct.c_void_p()
        _check(_LIB.tdmps_mps_from_dense(ctx.h, L, n_up + n_dn, n_up - n_dn, _dp(v), v.size, int(min(Dmax, 2 ** 31 - 1)),
                                         float(svd_cutoff), ct.byref(out)))
        return cls(out, L)

    def save(self, path):
        _check(_LIB.tdmps_mps_save(self.h, os.fsencode(path)))

    @classmethod
    def load(cls, ctx, path):
        out = ct.c_void_p()
        _check(_LIB.tdmps_mps_load(ctx.h, os.fsencode(path), ct.byref(out)))
        with open(path, "rb") as f:  # chain length from the documented file header
            L = int(np.frombuffer(f.read(12)[8:], dtype="<i4")[0])
        return cls(out, L)

    def sectors(self):
        tot = ct.c_int64()
        _check(_LIB.tdmps_mps_sectors(self.h, None, None, ct.byref(tot)))
        nsec = np.zeros(self.L + 1, dtype=np.int32)
        sec = np.zeros(3 * tot.value, dtype=np.int32)
        _check(_LIB.tdmps_mps_sectors(self.h, nsec.ctypes.data_as(_I32), sec.ctypes.data_as(_I32), ct.byref(tot)))
        out, k = [], 0
        for n in nsec:
            out.append([tuple(int(v) for v in sec[3 * (k + j):3 * (k + j) + 3]) for j in range(n)])
            k += n
        return out

    def get_blocks(self):
        n = ct.c_int64()
        _check(_LIB.tdmps_mps_get_blocks(self.h, None, ct.byref(n)))
        out = np.zeros(n.value)
        _check(_LIB.tdmps_mps_get_blocks(self.h, _dp(out), ct.byref(n)))
        return out.view(np.complex128)

    def to_dense(self):
        n = 4 ** self.L
        out = np.zeros(2 * n)
        _check(_LIB.tdmps_mps_to_dense(self.h, _dp(out), 2 * n))
        return out.view(np.complex128)

    def copy(self):
        out = ct.c_void_p()
        _check(_LIB.tdmps_mps_copy(self.h, ct.byref(out)))
        return MPS(out, self.L)

    def bond_dims(self):
        out = np.zeros(self.L + 1, dtype=np.int32)
        _check(_LIB.tdmps_mps_bond_dims(self.h, out.ctypes.data_as(_I32)))
        return out

    def scale(self, alpha):
        a = _cplx(alpha)
        _check(_LIB.tdmps_mps_scale(self.h, _dp(a)))

    def close(self):
        if self.h:
            _check(_LIB.tdmps_mps_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def overlap(a, b):
    out = np.zeros(2)
    _check(_LIB.tdmps_mps_overlap(a.h, b.h, _dp(out)))
    return complex(out[0], out[1])


def expect(op, bra, ket):
    out = np.zeros(2)
    _check(_LIB.tdmps_mps_expect(op.h, bra.h, ket.h, _dp(out)))
    return complex(out[0], out[1])


def _terms(terms):
    beta = np.array([x for b, _ in terms for x in _cplx(b)], dtype=np.float64)
    arr = (ct.c_void_p * max(1, len(terms)))(*[p.h.value if hasattr(p.h, "value") else p.h for _, p in terms])
    return beta, arr


def apply_H(H, alpha, psi, terms=(), params=None):
    params = params or fit_params()
    a = _cplx(alpha)
    beta, arr = _terms(terms)
    out, info = ct.c_void_p(), FitInfo()
    _check(_LIB.tdmps_mps_apply_H(H.h, _dp(a), psi.h, len(terms), _dp(beta) if len(terms) else None,
                                  ct.cast(arr, _PP), ct.byref(params), ct.byref(out), ct.byref(info)))
    return MPS(out, psi.L), info


def compress(terms, params=None):
    params = params or fit_params()
    beta, arr = _terms(terms)
    out, info = ct.c_void_p(), FitInfo()
    _check(_LIB.tdmps_mps_compress(len(terms), _dp(beta), ct.cast(arr, _PP), ct.byref(params), ct.byref(out),
                                   ct.byref(info)))
    return MPS(out, terms[0][1].L), info


def fiedler_order(h, eri=None):
    """Orbital permutation (new position -> old orbital) from the Fiedler vector of the
    coupling |h_ij| + |(ij|ji)|."""
    load()
    L = h.shape[0]
    h = np.ascontiguousarray(h, dtype=np.float64)
    e = None if eri is None else np.ascontiguousarray(eri, dtype=np.float64)
    perm = np.zeros(L, dtype=np.int32)
    _check(_LIB.tdmps_fiedler_order(L, _dp(h), None if e is None else e.ctypes.data_as(ct.c_void_p),
                                    perm.ctypes.data_as(_I32)))
    return perm


def permute_integrals(h, eri, perm):
    """Integrals in the new orbital order: h'[k, l] = h[perm[k], perm[l]], likewise eri."""
    p = np.asarray(perm)
    return h[np.ix_(p, p)], eri[np.ix_(p, p, p, p)]


def annihilate(psi, site, spin):
    """c_{site, spin} psi (spin 0 = up, 1 = down), exact."""
    out = ct.c_void_p()
    _check(_LIB.tdmps_mps_annihilate(psi.h, int(site), int(spin), ct.byref(out)))
    return MPS(out, psi.L)


def krylov_ground(H, psi, m, restarts, params=None):
    """Ground state by restarted Krylov iterations: (state, energy)."""
    params = params or fit_params()
    out, e = ct.c_void_p(), np.zeros(1)
    _check(_LIB.tdmps_krylov_ground(H.h, psi.h, int(m), int(restarts), ct.byref(params), ct.byref(out), _dp(e)))
    return MPS(out, psi.L), float(e[0])


def one_rdm(psi):
    """gamma_pq = sum_s <psi|a+_{ps} a_{qs}|psi> / <psi|psi> as an (L, L) complex array."""
    g = np.zeros(2 * psi.L * psi.L)
    _check(_LIB.tdmps_mps_one_rdm(psi.h, _dp(g)))
    return g.view(np.complex128).reshape(psi.L, psi.L)


def krylov_step(H, psi, dt, m, orthogonal=True, params=None):
    params = params or fit_params()
    N = np.zeros(2 * m * m)
    Hm = np.zeros(2 * m * m)
    out = ct.c_void_p()
    _check(_LIB.tdmps_krylov_step(H.h, psi.h, float(dt), m, KRYLOV_ORTHO if orthogonal else KRYLOV_NONORTHO,
                                  ct.byref(params), ct.byref(out), _dp(N), _dp(Hm)))
    return MPS(out, psi.L), N.view(np.complex128).reshape(m, m), Hm.view(np.complex128).reshape(m, m)


def rk4_step(H_t, psi, dt, params=None, H_mid=None, H_t1=None):
    params = params or fit_params()
    out, info = ct.c_void_p(), FitInfo()
    _check(_LIB.tdmps_rk4_step(H_t.h, (H_mid or H_t).h, (H_t1 or H_t).h, psi.h, float(dt), ct.byref(params),
                               ct.byref(out), ct.byref(info)))
    return MPS(out, psi.L), info


class Heff:
    """Two-site effective Hamiltonian at bond (site, site+1) between bra and ket."""

    def __init__(self, H, bra, ket, site, precision=FP64):
        out = ct.c_void_p()
        _check(_LIB.tdmps_heff_create(H.h, bra.h, ket.h, site, precision, ct.byref(out)))
        self.h = out

    def layout(self, which):
        """which = 0 (ket) or 1 (bra): (total doubles, blocks array of shape (n, 9))."""
        tot, nb = ct.c_int64(), ct.c_int64()
        _check(_LIB.tdmps_heff_layout(self.h, which, ct.byref(tot), ct.byref(nb), None))
        blocks = np.zeros(9 * nb.value, dtype=np.int32)
        _check(_LIB.tdmps_heff_layout(self.h, which, ct.byref(tot), ct.byref(nb), blocks.ctypes.data_as(_I32)))
        return tot.value, blocks.reshape(-1, 9)

    def apply(self, in_ptr, out_ptr):
        _check(_LIB.tdmps_heff_apply(self.h, ct.c_void_p(in_ptr), ct.c_void_p(out_ptr)))

    def apply_noalloc(self, in_ptr, out_ptr):
        """The same product in the library's fixed device scratch (no allocation)."""
        _check(_LIB.tdmps_heff_apply_noalloc(self.h, ct.c_void_p(in_ptr), ct.c_void_p(out_ptr)))

    def set_precision(self, precision):
        _check(_LIB.tdmps_heff_set_precision(self.h, int(precision)))

    def flops(self):
        f = ct.c_double()
        _check(_LIB.tdmps_heff_flops(self.h, ct.byref(f)))
        return f.value

    def close(self):
        if self.h:
            _check(_LIB.tdmps_heff_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class BlockLayout:
    """Helper to address panel-layout blocks of the heff two-site tensors on the host."""
    blocks: np.ndarray

    def offset(self, b):
        row = self.blocks[b]
        return (int(row[6]) | (int(row[7]) << 31)) // 2


class Trajectory:
    """Field-driven RK4 run keeping checkpoints; .value = D, .backward() = dD/d(amplitude)."""

    def __init__(self, H0, h0, m, mu, psi0, amplitude, omega, t_center, width, dt, nsteps, checkpoint_every=20,
                 params=None):
        params = params or fit_params()
        h0 = np.ascontiguousarray(h0, dtype=np.float64)
        m = np.ascontiguousarray(m, dtype=np.float64)
        pulse = Pulse(float(amplitude), float(omega), float(t_center), float(width))
        out, val = ct.c_void_p(), ct.c_double()
        _check(_LIB.tdmps_pulse_forward(H0.h, _dp(h0), _dp(m), mu.h, psi0.h, ct.byref(pulse), float(dt), int(nsteps),
                                        int(checkpoint_every), ct.byref(params), ct.byref(out), ct.byref(val)))
        self.h = out
        self.value = val.value

    def backward(self):
        g = ct.c_double()
        _check(_LIB.tdmps_pulse_backward(self.h, ct.byref(g)))
        return g.value

    def __del__(self):
        if getattr(self, "h", None) and _LIB is not None:
            _LIB.tdmps_traj_destroy(self.h)
            self.h = None
