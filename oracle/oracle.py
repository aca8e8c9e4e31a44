"""ctypes front end of the plain-C FP64 oracle (``snap_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
the benchmark call this module; the product path never does.  It imports nothing
from the product package.

Arrays follow the layout of the library boundary: positions, momenta and forces
are SoA ``float64[3, N]``; one periodic orthorhombic system per call.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "snap_oracle.c")
_LIB = os.path.join(_HERE, "libsnaporacle.so")
_lib = None

KB = 8.617333262145179e-5        # Boltzmann constant, eV/K
MVV2E = 1.0364269652680506e-4    # eV per amu*A^2/ps^2


def build_oracle(force=False):
    """Compile the oracle with gcc (plain IEEE FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build_oracle()
        L = C.CDLL(_LIB)
        d, i, u64, i64 = C.c_double, C.c_int, C.c_uint64, C.c_int64
        P = C.c_void_p
        L.ora_cg.restype = d
        L.ora_cg.argtypes = [i] * 6
        L.ora_wigner.restype = None
        L.ora_wigner.argtypes = [i, d, d, d, d, P]
        L.ora_snap_ncoeff.restype = i
        L.ora_snap_ncoeff.argtypes = [i]
        L.ora_neighbors.restype = i
        L.ora_neighbors.argtypes = [i, P, P, d, i, P, P]
        L.ora_snap_compute.restype = d
        L.ora_snap_compute.argtypes = [i, d, d, d, P, i, P, P, i, P, P, P, P, i, P, P]
        L.ora_snap_uy.restype = i
        L.ora_snap_uy.argtypes = [i, d, d, d, P, i, P, P, i, P, P]
        L.ora_fs_compute.restype = d
        L.ora_fs_compute.argtypes = [d, d, d, d, d, d, i, P, P, P, P]
        L.ora_philox4x64_10.restype = None
        L.ora_philox4x64_10.argtypes = [P, P, P]
        L.ora_gauss3.restype = None
        L.ora_gauss3.argtypes = [u64, u64, u64, u64, P]
        L.ora_gauss3t.restype = None
        L.ora_gauss3t.argtypes = [u64, u64, u64, u64, u64, P]
        L.ora_bbk.restype = i
        L.ora_bbk.argtypes = ([i, i, d, d, d, P, d, d, d, d, d, d, i, i, P, d, d, d, d, d, d,
                               u64, u64, i64, P, i, P, P, P, P, P])
        L.ora_set_threads.restype = i
        L.ora_set_threads.argtypes = [i]
        L.ora_langevin.restype = i
        L.ora_langevin.argtypes = ([i, i, d, d, d, P, d, d, d, d, d, d, i, i, P, d, d, d, d,
                                    u64, u64, i64, i, P, P, P, P, P])
        _lib = L
    return _lib


def set_threads(n):
    """Threads of the oracle's OpenMP loops (n <= 0 leaves them); returns the count in effect."""
    return lib().ora_set_threads(int(n))


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------------------
def cg(n1, k1, n2, k2, n, k):
    return lib().ora_cg(n1, k1, n2, k2, n, k)


def wigner(n, a, b):
    out = np.zeros(2 * (n + 1) ** 2)
    lib().ora_wigner(n, a.real, a.imag, b.real, b.imag, _p(out))
    return (out[0::2] + 1j * out[1::2]).reshape(n + 1, n + 1)


def ncoeff(J):
    return lib().ora_snap_ncoeff(J)


def neighbors(x, box, rcut, maxn=64):
    x = _c64(x)
    N = x.shape[1]
    cnt = np.zeros(N, np.int32)
    lst = np.full((N, maxn), -1, np.int32)
    rc = lib().ora_neighbors(N, _p(x), _p(_c64(box)), rcut, maxn, _p(cnt), _p(lst))
    if rc != 0:
        raise ValueError("neighbour list overflow")
    return cnt, lst


def snap_compute(x, box, J, beta, rcut=4.73, rfac0=0.99363, rmin0=0.0, route=0, maxn=64,
                 want_dedr=False):
    """SNAP energy and forces of one system.  route 0 = adjoint, 1 = direct.
    Returns dict(E, f[3,N], e_atom[N], B[N,K] and optionally dedr[N,maxn,3], count, list)."""
    x = _c64(x)
    N = x.shape[1]
    K = ncoeff(J)
    beta = _c64(beta)
    assert beta.shape == (K + 1,)
    f = np.zeros((3, N))
    ea = np.zeros(N)
    B = np.zeros((N, K))
    dedr = np.zeros((N, maxn, 3)) if want_dedr else None
    cnt = np.zeros(N, np.int32)
    lst = np.full((N, maxn), -1, np.int32)
    E = lib().ora_snap_compute(J, rcut, rfac0, rmin0, _p(beta), N, _p(x), _p(_c64(box)), route,
                               _p(f), _p(ea), _p(B), _p(dedr), maxn, _p(cnt), _p(lst))
    if not np.isfinite(E):
        raise ValueError("neighbour list overflow")
    out = dict(E=E, f=f, e_atom=ea, B=B, count=cnt, list=lst)
    if want_dedr:
        out["dedr"] = dedr
    return out


def snap_uy(x, box, J, beta, rcut=4.73, rfac0=0.99363, rmin0=0.0, maxn=64, want_y=True):
    """Per-atom density u and adjoint Y, full storage, as lists of [N, n+1, n+1] arrays."""
    x = _c64(x)
    N = x.shape[1]
    tot = sum((n + 1) ** 2 for n in range(J + 1))
    u = np.zeros((N, 2 * tot))
    y = np.zeros((N, 2 * tot)) if want_y else None
    rc = lib().ora_snap_uy(J, rcut, rfac0, rmin0, _p(_c64(beta)), N, _p(x), _p(_c64(box)), maxn,
                           _p(u), _p(y))
    if rc != 0:
        raise ValueError("neighbour list overflow")

    def split(a):
        c = a[:, 0::2] + 1j * a[:, 1::2]
        out, o = [], 0
        for n in range(J + 1):
            out.append(c[:, o:o + (n + 1) ** 2].reshape(N, n + 1, n + 1))
            o += (n + 1) ** 2
        return out
    return split(u), (split(y) if want_y else None)


def fs_compute(x, box, fs):
    """Finnis-Sinclair energy and forces.  fs = dict(A, d, c, c0, c1, c2)."""
    x = _c64(x)
    N = x.shape[1]
    f = np.zeros((3, N))
    ea = np.zeros(N)
    E = lib().ora_fs_compute(fs["A"], fs["d"], fs["c"], fs["c0"], fs["c1"], fs["c2"], N, _p(x),
                             _p(_c64(box)), _p(f), _p(ea))
    return dict(E=E, f=f, e_atom=ea)


def philox4x64_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, np.uint64)
    lib().ora_philox4x64_10(_p(c), _p(k), _p(out))
    return out


def gauss3(seed, noise_id, step, atom):
    g = np.zeros(3)
    lib().ora_gauss3(seed, noise_id, step & 0xFFFFFFFFFFFFFFFF, atom, _p(g))
    return g


POT_FS, POT_FS_SNAP, POT_NONE = 0, 1, 2


def langevin(x, p, box, *, potential, nsteps, dt, gamma, mass, T, seed, noise_id, step0,
             snap=None, fs=None, maxn=64, want_traj=False):
    """BAOAB steps of one system (positions and momenta are copied, not modified).
    snap = dict(J, beta, rcut, rfac0, rmin0); fs = dict(A, d, c, c0, c1, c2).
    Returns dict(x, p, f[, traj_x, traj_p] with traj_* of shape [nsteps+1, 3, N])."""
    x = _c64(x).copy()
    p = _c64(p).copy()
    N = x.shape[1]
    snap = snap or dict(J=0, beta=np.zeros(1), rcut=4.73, rfac0=0.99363, rmin0=0.0)
    fs = fs or dict(A=0, d=0, c=0, c0=0, c1=0, c2=0)
    beta = _c64(snap["beta"])
    f = np.zeros((3, N))
    tx = np.zeros((nsteps + 1, 3, N)) if want_traj else None
    tp = np.zeros((nsteps + 1, 3, N)) if want_traj else None
    rc = lib().ora_langevin(potential, snap["J"], snap.get("rcut", 4.73), snap.get("rfac0", 0.99363),
                            snap.get("rmin0", 0.0), _p(beta), fs["A"], fs["d"], fs["c"], fs["c0"],
                            fs["c1"], fs["c2"], maxn, N, _p(_c64(box)), dt, gamma, mass, T, seed,
                            noise_id, step0, nsteps, _p(x), _p(p), _p(f), _p(tx), _p(tp))
    if rc != 0:
        raise FloatingPointError("non-finite energy or neighbour overflow in oracle Langevin run")
    out = dict(x=x, p=p, f=f)
    if want_traj:
        out["traj_x"] = tx
        out["traj_p"] = tp
    return out


def gauss3t(seed, noise_id, step, atom, tag):
    g = np.zeros(3)
    lib().ora_gauss3t(seed, noise_id, step & 0xFFFFFFFFFFFFFFFF, atom, tag, _p(g))
    return g


def bbk(x, p, box, *, potential, nsteps, dt, gamma, mass, T, cT=(1.0, 1.0), seed=0, noise_id=0, step0=0,
        G=None, snap=None, fs=None, maxn=64, want_traj=False):
    """One application of nsteps iterates of the paper's modified BBK scheme (eq:scheme_debut,
    eq:scheme; with cT = (C_0, C_l>=1) the temperature schedule of eq:scheme_corrected_debut,
    eq:scheme_corrected) to one system; inputs are copied.  G: optional [nsteps+1, 3, N]
    Gaussians G_0..G_L (else drawn from Philox, see ora_bbk).  Returns dict(x, p, f[, traj_x,
    traj_p]) with traj_* of shape [nsteps+1, 3, N] (q_l, p_l)."""
    x = _c64(x).copy()
    p = _c64(p).copy()
    N = x.shape[1]
    snap = snap or dict(J=0, beta=np.zeros(1), rcut=4.73, rfac0=0.99363, rmin0=0.0)
    fs = fs or dict(A=0, d=0, c=0, c0=0, c1=0, c2=0)
    beta = _c64(snap["beta"])
    if G is not None:
        G = _c64(G)
        if G.shape != (nsteps + 1, 3, N):
            raise ValueError("G must have shape (nsteps + 1, 3, N)")
    f = np.zeros((3, N))
    tx = np.zeros((nsteps + 1, 3, N)) if want_traj else None
    tp = np.zeros((nsteps + 1, 3, N)) if want_traj else None
    rc = lib().ora_bbk(potential, snap["J"], snap.get("rcut", 4.73), snap.get("rfac0", 0.99363),
                       snap.get("rmin0", 0.0), _p(beta), fs["A"], fs["d"], fs["c"], fs["c0"], fs["c1"], fs["c2"],
                       maxn, N, _p(_c64(box)), dt, gamma, mass, T, float(cT[0]), float(cT[1]), seed, noise_id,
                       step0, _p(G), nsteps, _p(x), _p(p), _p(f), _p(tx), _p(tp))
    if rc != 0:
        raise FloatingPointError("non-finite energy or neighbour overflow in oracle BBK run")
    out = dict(x=x, p=p, f=f)
    if want_traj:
        out["traj_x"] = tx
        out["traj_p"] = tp
    return out
