"""Thin Python binding of the snapmd C ABI (include/snapmd.h): argument marshalling only.

Every computation runs in the HIP kernels of ``libsnapmd.so``; this module converts
torch tensors (device memory, current HIP stream) and NumPy arrays (small host
parameter arrays) into the C structs and checks return codes.  There is no CPU
fallback: if the library is missing, importing the entry points raises.
"""
import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsnapmd.so")

OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED, ENONFINITE, EOVERFLOW = 0, -1, -2, -3, -4, -5, -6
MAX_NEIGH = 64
ACCUMULATE = 1
POT_FS, POT_FS_SNAP = 0, 1


class SnapmdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("snapmd error %d: %s" % (code, msg))
        self.code = code


class Batch(C.Structure):
    _fields_ = [("n_sys", C.c_int32), ("offset", C.POINTER(C.c_int32)), ("box", C.POINTER(C.c_double))]


class Snap(C.Structure):
    _fields_ = [("twojmax", C.c_int32), ("rcut", C.c_double), ("rfac0", C.c_double), ("rmin0", C.c_double),
                ("n_coeff", C.c_int32), ("beta", C.POINTER(C.c_double))]


class Fs(C.Structure):
    _fields_ = [("A", C.c_double), ("d", C.c_double), ("c", C.c_double), ("c0", C.c_double),
                ("c1", C.c_double), ("c2", C.c_double)]


class Langevin(C.Structure):
    _fields_ = [("dt", C.c_double), ("gamma", C.c_double), ("mass", C.c_double),
                ("T_sys", C.POINTER(C.c_double)), ("seed", C.c_uint64),
                ("step0_sys", C.POINTER(C.c_int64)), ("noise_id_sys", C.POINTER(C.c_int32)),
                ("scheme", C.c_int32), ("bbk_c0", C.c_double), ("bbk_c1", C.c_double)]


class KShape(C.Structure):
    _fields_ = [("density_acc", C.c_int32), ("dedr_stage_atoms", C.c_int32), ("adjoint_waves", C.c_int32),
                ("density_parts", C.c_int32)]


# compiled variants of each kernel-shape field (twojmax <= 8)
SHAPE_CHOICES = {"density_acc": (45, 28, 21), "dedr_stage_atoms": (5, 3, 0), "adjoint_waves": (12, 8),
                 "density_parts": (1, 2, 0)}
DEFAULT_SHAPE = (45, 0, 12, 0)


class ParaLog(C.Structure):
    _fields_ = [("max_log", C.c_int32), ("n_log", C.POINTER(C.c_int32)), ("n_in", C.POINTER(C.c_int32)),
                ("n_fi", C.POINTER(C.c_int32)), ("n_fi_after", C.POINTER(C.c_int32)),
                ("delta", C.POINTER(C.c_double))]


_lib = None


def lib():
    """Load libsnapmd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("snapmd HIP library not built: run `python -m paper_2212_10508_amd.build` "
                          "(expected %s)" % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    P, i32, u32, d = C.c_void_p, C.c_int32, C.c_uint32, C.c_double
    L.snapmd_create.argtypes = [C.POINTER(P), C.c_int]
    L.snapmd_create.restype = C.c_int
    L.snapmd_destroy.argtypes = [P]
    L.snapmd_destroy.restype = None
    L.snapmd_last_error.argtypes = [P]
    L.snapmd_last_error.restype = C.c_char_p
    L.snapmd_sync.argtypes = [P, P]
    L.snapmd_sync.restype = C.c_int
    L.snap_forces.argtypes = [P, C.POINTER(Snap), C.POINTER(Batch), P, P, P, u32, P]
    L.snap_forces.restype = C.c_int
    L.snap_forces_noalloc.argtypes = [P, C.POINTER(Snap), C.POINTER(Batch), P, P, P, u32, P]
    L.snap_forces_noalloc.restype = C.c_int
    L.eam_forces.argtypes = [P, C.POINTER(Fs), C.POINTER(Batch), P, P, P, u32, P]
    L.eam_forces.restype = C.c_int
    L.langevin_steps.argtypes = [P, C.c_int, C.POINTER(Snap), C.POINTER(Fs), C.POINTER(Batch),
                                 C.POINTER(Langevin), i32, P, P, P, P]
    L.langevin_steps.restype = C.c_int
    L.parareal_iterate.argtypes = [P, C.POINTER(Snap), C.POINTER(Fs), C.POINTER(Batch), C.POINTER(Langevin),
                                   i32, C.POINTER(i32), C.POINTER(i32), i32, P, P, P, P, d, C.POINTER(d), P]
    L.parareal_iterate.restype = C.c_int
    L.parareal_iterate_async.argtypes = [P, C.POINTER(Snap), C.POINTER(Fs), C.POINTER(Batch), C.POINTER(Langevin),
                                         i32, i32, i32, i32, P, P, P, P, d, P]
    L.parareal_iterate_async.restype = C.c_int
    L.snapmd_parareal_collect.argtypes = [P, C.POINTER(d), C.POINTER(i32), P]
    L.snapmd_parareal_collect.restype = C.c_int
    L.parareal_adaptive.argtypes = [P, C.POINTER(Snap), C.POINTER(Fs), C.POINTER(Batch), C.POINTER(Langevin),
                                    i32, i32, i32, d, d, i32, i32, P, P, C.POINTER(ParaLog), C.POINTER(i32),
                                    C.POINTER(i32), P]
    L.parareal_adaptive.restype = C.c_int
    L.snap_beta_grad.argtypes = [P, C.POINTER(Snap), C.POINTER(Batch), P, P, P, P, P]
    L.snap_beta_grad.restype = C.c_int
    L.snapmd_bispectrum.argtypes = [P, C.POINTER(Snap), C.POINTER(Batch), P, P, P]
    L.snapmd_bispectrum.restype = C.c_int
    L.snapmd_use_graphs.argtypes = [P, C.c_int]
    L.snapmd_use_graphs.restype = C.c_int
    L.snapmd_profile.argtypes = [P, C.c_int]
    L.snapmd_profile.restype = C.c_int
    L.snapmd_profile_read.argtypes = [P, C.c_int, C.POINTER(d), C.POINTER(C.c_int64)]
    L.snapmd_profile_read.restype = C.c_int
    L.snapmd_pair_count.argtypes = [P, C.POINTER(C.c_int64)]
    L.snapmd_pair_count.restype = C.c_int
    L.snapmd_ws_sites.argtypes = [P, C.POINTER(Batch), P, d, P, P, i32, P]
    L.snapmd_ws_sites.restype = C.c_int
    L.snapmd_relax.argtypes = [P, C.c_int, C.POINTER(Snap), C.POINTER(Fs), C.POINTER(Batch), P, i32, d, d, d,
                               C.POINTER(d), C.POINTER(i32), P]
    L.snapmd_relax.restype = C.c_int
    L.snapmd_set_kernel_shape.argtypes = [P, i32, C.POINTER(KShape)]
    L.snapmd_set_kernel_shape.restype = C.c_int
    L.snapmd_get_kernel_shape.argtypes = [P, i32, C.POINTER(KShape)]
    L.snapmd_get_kernel_shape.restype = C.c_int
    L.snapmd_set_coarse_fs.argtypes = [P, C.POINTER(Fs)]
    L.snapmd_set_coarse_fs.restype = C.c_int
    L.snapmd_set_coarse_snap.argtypes = [P, C.POINTER(Snap)]
    L.snapmd_set_coarse_snap.restype = C.c_int
    L.snapmd_set_chunk_plan.argtypes = [P, C.POINTER(i32), i32]
    L.snapmd_set_chunk_plan.restype = C.c_int
    L.snapmd_chunk_plan.argtypes = [P, i32, i32, C.POINTER(i32), C.POINTER(i32)]
    L.snapmd_chunk_plan.restype = C.c_int
    L.snapmd_set_sweep_workgroups.argtypes = [P, i32]
    L.snapmd_set_sweep_workgroups.restype = C.c_int
    L.snapmd_set_fine_streams.argtypes = [P, i32]
    L.snapmd_set_fine_streams.restype = C.c_int
    L.snapmd_sweep_workgroups.argtypes = [P, i32, C.POINTER(i32)]
    L.snapmd_sweep_workgroups.restype = C.c_int
    _lib = L
    return L


# ----------------------------------------------------------------------------
# marshalling helpers
# ----------------------------------------------------------------------------
def _dev(t, name, shape=None, dtype=torch.float64):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) torch tensor" % name)
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError("%s must be a contiguous %s tensor" % (name, dtype))
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s (got %s)" % (name, tuple(shape), tuple(t.shape)))
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class _Keep:
    """Holds the NumPy arrays referenced by a C struct for the duration of a call."""

    def __init__(self):
        self.refs = []

    def arr(self, a, dtype, ctype):
        a = np.ascontiguousarray(a, dtype=dtype)
        self.refs.append(a)
        return a.ctypes.data_as(C.POINTER(ctype))


def make_batch(keep, offset, box):
    offset = np.asarray(offset, np.int32)
    box = np.asarray(box, np.float64).reshape(-1)
    return Batch(len(offset) - 1, keep.arr(offset, np.int32, C.c_int32), keep.arr(box, np.float64, C.c_double))


def make_snap(keep, J, beta, rcut=4.73, rfac0=0.99363, rmin0=0.0):
    beta = np.asarray(beta, np.float64)
    return Snap(J, rcut, rfac0, rmin0, len(beta) - 1, keep.arr(beta, np.float64, C.c_double))


def make_fs(fs):
    return Fs(fs["A"], fs["d"], fs["c"], fs["c0"], fs["c1"], fs["c2"])


SCHEMES = {"baoab": 0, "bbk": 1}


def make_langevin(keep, n_sys, dt, gamma, mass, T, seed, step0, noise_id, scheme="baoab", cT=(1.0, 1.0)):
    T = np.broadcast_to(np.asarray(T, np.float64), (n_sys,))
    step0 = np.broadcast_to(np.asarray(step0, np.int64), (n_sys,))
    noise_id = np.broadcast_to(np.asarray(noise_id, np.int32), (n_sys,))
    if scheme not in SCHEMES:
        raise ValueError("scheme must be one of %s" % sorted(SCHEMES))
    return Langevin(dt, gamma, mass, keep.arr(T, np.float64, C.c_double), seed,
                    keep.arr(step0, np.int64, C.c_int64), keep.arr(noise_id, np.int32, C.c_int32),
                    SCHEMES[scheme], float(cT[0]), float(cT[1]))


# ----------------------------------------------------------------------------
# context and entry points
# ----------------------------------------------------------------------------
def check_windows(n_in, n_fi, n_slots, n_sys):
    """Windows of parareal_iterate: 0 <= n_in <= n_fi <= n_slots - 1 per system (the state
    arrays hold slots 0 .. n_slots - 1), non-empty for a single system."""
    n_in = np.asarray(n_in).reshape(-1)
    n_fi = np.asarray(n_fi).reshape(-1)
    if n_in.shape != (n_sys,) or n_fi.shape != (n_sys,):
        raise ValueError("n_in and n_fi need one entry per system (%d)" % n_sys)
    for r in range(n_sys):
        a, b = int(n_in[r]), int(n_fi[r])
        if a < 0 or b < a or b > n_slots - 1 or (n_sys == 1 and a == b):
            raise ValueError("system %d: need 0 <= n_in < n_fi <= n_slots - 1 (got %d, %d with %d slots)"
                             % (r, a, b, n_slots))


class Context:
    """A snapmd context on one HIP device (owns the library workspace)."""

    def __init__(self, device=0):
        L = lib()
        h = C.c_void_p()
        rc = L.snapmd_create(C.byref(h), int(device))
        if rc != OK:
            raise SnapmdError(rc, "snapmd_create(%d) failed" % device)
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            lib().snapmd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != OK:
            raise SnapmdError(rc, lib().snapmd_last_error(self.h).decode())

    def sync(self, stream=None):
        self._check(lib().snapmd_sync(self.h, _stream(stream)))

    # -- forces ------------------------------------------------------------
    def snap_forces(self, x, offset, box, J, beta, f=None, e_atom=None, accumulate=False, rcut=4.73,
                    rfac0=0.99363, rmin0=0.0, stream=None):
        N = int(offset[-1])
        k = _Keep()
        b, s = make_batch(k, offset, box), make_snap(k, J, beta, rcut, rfac0, rmin0)
        if f is None:
            f = torch.empty((3, N), dtype=torch.float64, device=x.device)
        self._check(lib().snap_forces(self.h, C.byref(s), C.byref(b), _dev(x, "x", (3, N)), _dev(f, "f", (3, N)),
                                      _dev(e_atom, "e_atom", (N,)), ACCUMULATE if accumulate else 0,
                                      _stream(stream)))
        return f

    def snap_forces_noalloc(self, x, offset, box, J, beta, f, e_atom=None, accumulate=False, rcut=4.73,
                            rfac0=0.99363, rmin0=0.0, stream=None):
        """snap_forces without any device allocation (f is required; at most
        SNAPMD_NOALLOC_MAX_ATOMS atoms)."""
        N = int(offset[-1])
        k = _Keep()
        b, s = make_batch(k, offset, box), make_snap(k, J, beta, rcut, rfac0, rmin0)
        self._check(lib().snap_forces_noalloc(self.h, C.byref(s), C.byref(b), _dev(x, "x", (3, N)),
                                              _dev(f, "f", (3, N)), _dev(e_atom, "e_atom", (N,)),
                                              ACCUMULATE if accumulate else 0, _stream(stream)))
        return f

    def eam_forces(self, x, offset, box, fs, f=None, e_atom=None, accumulate=False, stream=None):
        N = int(offset[-1])
        k = _Keep()
        b, p = make_batch(k, offset, box), make_fs(fs)
        if f is None:
            f = torch.empty((3, N), dtype=torch.float64, device=x.device)
        self._check(lib().eam_forces(self.h, C.byref(p), C.byref(b), _dev(x, "x", (3, N)), _dev(f, "f", (3, N)),
                                     _dev(e_atom, "e_atom", (N,)), ACCUMULATE if accumulate else 0,
                                     _stream(stream)))
        return f

    def bispectrum(self, x, offset, box, J, beta, rcut=4.73, rfac0=0.99363, rmin0=0.0, stream=None):
        N = int(offset[-1])
        k = _Keep()
        b, s = make_batch(k, offset, box), make_snap(k, J, beta, rcut, rfac0, rmin0)
        B = torch.empty((len(beta) - 1, N), dtype=torch.float64, device=x.device)
        self._check(lib().snapmd_bispectrum(self.h, C.byref(s), C.byref(b), _dev(x, "x", (3, N)),
                                            _dev(B, "B"), _stream(stream)))
        return B

    # -- dynamics ----------------------------------------------------------
    def langevin_steps(self, potential, x, p, offset, box, n_steps, *, dt, gamma, mass, T, seed, step0,
                       noise_id, fs, J=None, beta=None, f_out=None, rcut=4.73, rfac0=0.99363, rmin0=0.0,
                       scheme="baoab", cT=(1.0, 1.0), stream=None):
        """scheme "bbk": one call is one application of n_steps iterates of the paper's
        scheme with temperature factors cT = (C_0, C_l>=1)."""
        N = int(offset[-1])
        S = len(offset) - 1
        k = _Keep()
        b = make_batch(k, offset, box)
        s = make_snap(k, J, beta, rcut, rfac0, rmin0) if potential == POT_FS_SNAP else None
        p_fs = make_fs(fs)
        lg = make_langevin(k, S, dt, gamma, mass, T, seed, step0, noise_id, scheme, cT)
        self._check(lib().langevin_steps(self.h, potential, C.byref(s) if s is not None else None,
                                         C.byref(p_fs), C.byref(b), C.byref(lg), int(n_steps),
                                         _dev(x, "x", (3, N)), _dev(p, "p", (3, N)),
                                         _dev(f_out, "f_out", (3, N)), _stream(stream)))

    def parareal_iterate(self, q_prev, p_prev, q_cur, p_cur, box, L, n_in, n_fi, delta_expl, *, dt, gamma,
                         mass, T, seed, noise_id, fs, J=None, beta=None, rcut=4.73, rfac0=0.99363, rmin0=0.0,
                         scheme="baoab", cT=(1.0, 1.0), stream=None):
        """One system (states [n_slots, 3, N]).  Returns (delta, n_fi_after).
        q_prev = p_prev = None: window initialisation."""
        N = q_cur.shape[2]
        d, nf = self.parareal_iterate_batch(q_prev, p_prev, q_cur, p_cur, [0, N], [box], L, [n_in], [n_fi],
                                            delta_expl, dt=dt, gamma=gamma, mass=mass, T=[T], seed=seed,
                                            noise_id=[noise_id], fs=fs, J=J, beta=beta, rcut=rcut, rfac0=rfac0,
                                            rmin0=rmin0, scheme=scheme, cT=cT, stream=stream)
        return float(d[0]), int(nf[0])

    def parareal_iterate_async(self, q_prev, p_prev, q_cur, p_cur, box, L, n_in, n_fi, delta_expl, *, dt, gamma,
                               mass, T, seed, noise_id, fs, J=None, beta=None, rcut=4.73, rfac0=0.99363, rmin0=0.0,
                               scheme="baoab", cT=(1.0, 1.0), stream=None):
        """parareal_iterate of one system, enqueued (pipelined with the previous iteration of
        the same window); its (delta, n_fi_after) come from parareal_collect()."""
        nslots, three, N = q_cur.shape
        check_windows(np.array([n_in], np.int32), np.array([n_fi], np.int32), nslots, 1)
        k = _Keep()
        b = make_batch(k, [0, N], [box])
        s = make_snap(k, J, beta, rcut, rfac0, rmin0) if beta is not None else None
        p_fs = make_fs(fs)
        lg = make_langevin(k, 1, dt, gamma, mass, [T], seed, 0, [noise_id], scheme, cT)
        shape = (nslots, 3, N)
        self._check(lib().parareal_iterate_async(
            self.h, C.byref(s) if s is not None else None, C.byref(p_fs), C.byref(b), C.byref(lg), int(L),
            int(n_in), int(n_fi), int(nslots),
            _dev(q_prev, "q_prev", shape) if q_prev is not None else None,
            _dev(p_prev, "p_prev", shape) if p_prev is not None else None,
            _dev(q_cur, "q_cur", shape), _dev(p_cur, "p_cur", shape), float(delta_expl), _stream(stream)))

    def parareal_collect(self, stream=None):
        """(delta, n_fi_after) of the oldest uncollected parareal_iterate_async call; its
        states are complete once this returns (`stream` waits for them)."""
        d = C.c_double(0.0)
        nf = C.c_int32(0)
        self._check(lib().snapmd_parareal_collect(self.h, C.byref(d), C.byref(nf), _stream(stream)))
        return d.value, nf.value

    def parareal_iterate_batch(self, q_prev, p_prev, q_cur, p_cur, offset, box, L, n_in, n_fi, delta_expl, *, dt,
                               gamma, mass, T, seed, noise_id, fs, J=None, beta=None, rcut=4.73, rfac0=0.99363,
                               rmin0=0.0, scheme="baoab", cT=(1.0, 1.0), stream=None):
        """Every system r of the batch (offset, box as for langevin_steps) on its own window
        [n_in[r], n_fi[r]]; states [n_slots, 3, offset[-1]] (system r in columns
        offset[r]:offset[r+1]).  T and noise_id per system (or one value for all).
        Returns (delta, n_fi_after) as numpy arrays.  q_prev = p_prev = None: window
        initialisation."""
        nslots, three, N = q_cur.shape
        R = len(offset) - 1
        n_in = np.asarray(n_in, dtype=np.int32).reshape(-1)
        n_fi = np.asarray(n_fi, dtype=np.int32).reshape(-1)
        check_windows(n_in, n_fi, nslots, R)
        if int(offset[-1]) != N:
            raise ValueError("offset[-1] = %d but the states hold %d atoms" % (int(offset[-1]), N))
        k = _Keep()
        b = make_batch(k, offset, box)
        s = make_snap(k, J, beta, rcut, rfac0, rmin0) if beta is not None else None
        p_fs = make_fs(fs)
        lg = make_langevin(k, R, dt, gamma, mass, T, seed, 0, noise_id, scheme, cT)
        nin_c = k.arr(n_in, np.int32, C.c_int32)
        nfi = np.ascontiguousarray(n_fi.copy())
        delta = np.zeros(R, np.float64)
        shape = (nslots, 3, N)
        self._check(lib().parareal_iterate(
            self.h, C.byref(s) if s is not None else None, C.byref(p_fs), C.byref(b), C.byref(lg), int(L), nin_c,
            nfi.ctypes.data_as(C.POINTER(C.c_int32)), int(nslots),
            _dev(q_prev, "q_prev", shape) if q_prev is not None else None,
            _dev(p_prev, "p_prev", shape) if p_prev is not None else None,
            _dev(q_cur, "q_cur", shape), _dev(p_cur, "p_cur", shape), float(delta_expl),
            delta.ctypes.data_as(C.POINTER(C.c_double)), _stream(stream)))
        return delta, nfi

    def parareal_adaptive(self, q, p, offset, box, N, L, delta_conv, delta_expl, *, dt, gamma, mass, T, seed,
                          noise_id, fs, J, beta, max_window=None, rounds_per_check=4, max_rounds=10000,
                          max_log=256, rcut=4.73, rfac0=0.99363, rmin0=0.0, stream=None):
        """The adaptive algorithm for every system of the batch, decided on the device.
        q, p: device [N+1, 3, offset[-1]] with the initial states in slot 0; on return they
        hold the converged trajectories.  Returns dict(logs (per system, one dict per
        iteration: n_in, n_fi, n_fi_after, delta), n_ad, kconv, rounds, checks)."""
        R = len(offset) - 1
        nt = int(offset[-1])
        k = _Keep()
        b = make_batch(k, offset, box)
        s = make_snap(k, J, beta, rcut, rfac0, rmin0)
        p_fs = make_fs(fs)
        lg = make_langevin(k, R, dt, gamma, mass, T, seed, 0, noise_id, "baoab")
        ML = int(max_log)
        n_log = np.zeros(R, np.int32)
        a_in = np.zeros(R * max(ML, 1), np.int32)
        a_fi = np.zeros_like(a_in)
        a_af = np.zeros_like(a_in)
        a_d = np.zeros(R * max(ML, 1), np.float64)
        ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
        lgs = ParaLog(ML, ip(n_log), ip(a_in), ip(a_fi), ip(a_af), a_d.ctypes.data_as(C.POINTER(C.c_double)))
        rounds, checks = C.c_int32(0), C.c_int32(0)
        shape = (int(N) + 1, 3, nt)
        self._check(lib().parareal_adaptive(
            self.h, C.byref(s), C.byref(p_fs), C.byref(b), C.byref(lg), int(L), int(N),
            int(max_window if max_window is not None else N), float(delta_conv), float(delta_expl),
            int(rounds_per_check), int(max_rounds), _dev(q, "q", shape), _dev(p, "p", shape), C.byref(lgs),
            C.byref(rounds), C.byref(checks), _stream(stream)))
        logs, n_ad, kconv = [], [], []
        for r in range(R):
            rows = [dict(n_in=int(a_in[r * ML + t]), n_fi=int(a_fi[r * ML + t]), n_fi_after=int(a_af[r * ML + t]),
                         delta=float(a_d[r * ML + t])) for t in range(min(int(n_log[r]), ML))]
            logs.append(rows)
            kc = []
            for t, row in enumerate(rows):
                if t == 0 or row["n_in"] != rows[t - 1]["n_in"]:
                    kc.append(0)
                kc[-1] += 1
            n_ad.append(len(kc))
            kconv.append(kc)
        return dict(logs=logs, n_ad=n_ad, kconv=kconv, rounds=rounds.value, checks=checks.value)

    # -- measurement ---------------------------------------------------------
    PROF_DEDR, PROF_ADJOINT, PROF_DENSITY, PROF_NEIGH = 0, 1, 2, 3

    def use_graphs(self, enable=True):
        """Replay captured hipGraphs of the Langevin launch sequences (default on)."""
        self._check(lib().snapmd_use_graphs(self.h, 1 if enable else 0))

    def profile(self, enable=True, every=1):
        """Record HIP events around every `every`-th launch of the SNAP kernels and the
        neighbour build (enable=False stops)."""
        self._check(lib().snapmd_profile(self.h, int(every) if enable else 0))

    def profile_read(self, kernel):
        """(total ms, launches) of HIP-event-timed launches of `kernel` since profile(True)."""
        ms = C.c_double(0.0)
        n = C.c_int64(0)
        self._check(lib().snapmd_profile_read(self.h, int(kernel), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def ws_sites(self, x, offset, box, a, stream=None):
        """Wigner-Seitz site of every atom on the bcc lattice of constant a, and the number
        of atoms of every site: (site int32 [N], occ int32 [n_sites]) device tensors."""
        N = int(offset[-1])
        box = np.asarray(box, np.float64).reshape(-1, 3)
        n_sites = int(sum(2 * np.prod(np.rint(b / a)) for b in box))
        site = torch.empty(N, dtype=torch.int32, device=x.device)
        occ = torch.empty(max(n_sites, 1), dtype=torch.int32, device=x.device)
        k = _Keep()
        b = make_batch(k, offset, box)
        self._check(lib().snapmd_ws_sites(self.h, C.byref(b), _dev(x, "x", (3, N)), float(a),
                                          _dev(site, "site", (N,), torch.int32),
                                          _dev(occ, "occ", None, torch.int32), int(occ.numel()), _stream(stream)))
        return site, occ[:n_sites]

    def relax(self, potential, x, offset, box, fs, J=None, beta=None, max_iter=5000, ftol=1e-4, alpha=0.01,
              dmax=0.02, rcut=4.73, rfac0=0.99363, rmin0=0.0, stream=None):
        """Steepest descent of the energy in place; returns (max |F| in eV/A, steps)."""
        N = int(offset[-1])
        k = _Keep()
        b = make_batch(k, offset, box)
        s = make_snap(k, J, beta, rcut, rfac0, rmin0) if potential == POT_FS_SNAP else None
        fm = C.c_double(0.0)
        its = C.c_int32(0)
        self._check(lib().snapmd_relax(self.h, potential, C.byref(s) if s is not None else None, C.byref(make_fs(fs)),
                                       C.byref(b), _dev(x, "x", (3, N)), int(max_iter), float(ftol), float(alpha),
                                       float(dmax), C.byref(fm), C.byref(its), _stream(stream)))
        return fm.value, its.value

    def set_coarse_snap(self, J=None, beta=None, rcut=4.73, rfac0=0.99363, rmin0=0.0):
        """Coarse propagator of parareal_iterate: Finnis-Sinclair + SNAP(J, beta) (the
        paper's strategy I), or Finnis-Sinclair alone with J=None."""
        if J is None:
            self._check(lib().snapmd_set_coarse_snap(self.h, None))
            return
        k = _Keep()
        s = make_snap(k, J, beta, rcut, rfac0, rmin0)
        self._check(lib().snapmd_set_coarse_snap(self.h, C.byref(s)))

    def set_kernel_shape(self, J, shape):
        """Kernel shape (density_acc, dedr_stage_atoms, adjoint_waves, density_parts) of the
        SNAP passes at twojmax J (None: the built-in shape; a shape of three values has
        density_parts 1; density_parts 0 splits the density pass of launches with fewer
        waves than the device has SIMDs)."""
        if shape is None:
            self._check(lib().snapmd_set_kernel_shape(self.h, int(J), None))
        else:
            v = [int(q) for q in shape]
            if len(v) == 3:
                v.append(1)
            if len(v) != 4:
                raise ValueError("a kernel shape has 3 or 4 values (got %d)" % len(v))
            ks = KShape(*v)
            self._check(lib().snapmd_set_kernel_shape(self.h, int(J), C.byref(ks)))

    def kernel_shape(self, J):
        ks = KShape()
        self._check(lib().snapmd_get_kernel_shape(self.h, int(J), C.byref(ks)))
        return (ks.density_acc, ks.dedr_stage_atoms, ks.adjoint_waves, ks.density_parts)

    def set_coarse_fs(self, fs):
        """Finnis-Sinclair parameters of the coarse propagator of parareal_iterate (a dict like
        the fs argument; None: the fs passed to each call)."""
        if fs is None:
            self._check(lib().snapmd_set_coarse_fs(self.h, None))
        else:
            p_fs = make_fs(fs)
            self._check(lib().snapmd_set_coarse_fs(self.h, C.byref(p_fs)))

    def set_chunk_plan(self, sizes):
        """Slab chunks of parareal_iterate for windows of sum(sizes) slabs (None or []:
        the built-in plan)."""
        sizes = list(sizes or [])
        arr = (C.c_int32 * max(len(sizes), 1))(*sizes)
        self._check(lib().snapmd_set_chunk_plan(self.h, arr, len(sizes)))

    def chunk_plan(self, S, N):
        """The chunks parareal_iterate uses for a window of S slabs of N atoms."""
        arr = (C.c_int32 * 64)()
        n = C.c_int32(0)
        self._check(lib().snapmd_chunk_plan(self.h, int(S), int(N), arr, C.byref(n)))
        return list(arr[:n.value])

    def set_sweep_workgroups(self, K):
        """Workgroups of the on-device coarse sweep in later parareal_iterate calls (0: the
        built-in choice)."""
        self._check(lib().snapmd_set_sweep_workgroups(self.h, int(K)))

    def set_fine_streams(self, n):
        """SNAP streams of a parareal iteration of one system in later calls (2: the odd slab
        chunks on a second stream beside the even ones; 1: all on the caller's stream)."""
        self._check(lib().snapmd_set_fine_streams(self.h, int(n)))

    def sweep_workgroups(self, N):
        """The sweep width a system of N atoms gets (0: one workgroup or host-driven)."""
        k = C.c_int32(0)
        self._check(lib().snapmd_sweep_workgroups(self.h, int(N), C.byref(k)))
        return k.value

    def pair_count(self):
        n = C.c_int64(0)
        self._check(lib().snapmd_pair_count(self.h, C.byref(n)))
        return n.value

    def snap_beta_grad(self, x, w, offset, box, J, beta, rcut=4.73, rfac0=0.99363, rmin0=0.0, stream=None):
        """Returns (dE/dbeta [K+1], sum_i w_i . dF_i/dbeta [K+1]) as device tensors."""
        N = int(offset[-1])
        K1 = len(beta)
        k = _Keep()
        b, s = make_batch(k, offset, box), make_snap(k, J, beta, rcut, rfac0, rmin0)
        dE = torch.empty(K1, dtype=torch.float64, device=x.device)
        gF = torch.empty(K1, dtype=torch.float64, device=x.device)
        self._check(lib().snap_beta_grad(self.h, C.byref(s), C.byref(b), _dev(x, "x", (3, N)),
                                         _dev(w, "w", (3, N)), _dev(dE, "dE"), _dev(gF, "gF"),
                                         _stream(stream)))
        return dE, gF


_default = {}


def context(device=0):
    """Process-wide context per device."""
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def snap_forces(x, offset, box, J, beta, **kw):
    return context(x.device.index or 0).snap_forces(x, offset, box, J, beta, **kw)


def eam_forces(x, offset, box, fs, **kw):
    return context(x.device.index or 0).eam_forces(x, offset, box, fs, **kw)


def langevin_steps(potential, x, p, offset, box, n_steps, **kw):
    return context(x.device.index or 0).langevin_steps(potential, x, p, offset, box, n_steps, **kw)


def parareal_iterate(q_prev, p_prev, q_cur, p_cur, box, L, n_in, n_fi, delta_expl, **kw):
    return context(q_cur.device.index or 0).parareal_iterate(q_prev, p_prev, q_cur, p_cur, box, L, n_in,
                                                             n_fi, delta_expl, **kw)


def snap_beta_grad(x, w, offset, box, J, beta, **kw):
    return context(x.device.index or 0).snap_beta_grad(x, w, offset, box, J, beta, **kw)
