"""CPU oracle for checkerboard Metropolis sweeps of the 2D Ising model.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this
package; only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may.  It shares no code with the GPU library.

Contents:
  - ``liboracle.so`` (from ``ising_oracle.c``): Philox4x32-10, thresholds,
    random/cold initial states, plain int8 sweeps, observables, threaded
    batches over replicas; (from ``cluster_oracle.c``) Swendsen-Wang and Wolff
    cluster steps; (from ``ising3d_oracle.c``) 3D sweeps.  This module is its
    ctypes front-end.
  - ``philox``: a second, pure-Python Philox4x32-10.
  - ``exact``: exact results (enumeration, transfer matrix, Kaufman torus
    partition function, Onsager energy and T_c, Yang magnetisation).
  - ``stats``: autocorrelation time, binned errors, chi-square helpers.
  - ``nn_ref``: float64 numpy reference of the block-proposal network.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

INIT_RANDOM, INIT_UP, INIT_DOWN = 0, 1, 2


class Desc(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32), ("J", ctypes.c_double),
                ("beta", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("replica", ctypes.c_uint32), ("init", ctypes.c_int32), ("rng", ctypes.c_int32)]


class Desc3(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32), ("Lz", ctypes.c_int32), ("init", ctypes.c_int32),
                ("J", ctypes.c_double), ("beta", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("replica", ctypes.c_uint32), ("rng", ctypes.c_int32)]


_lib = None


def lib():
    """Load liboracle.so, building it with gcc first if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from oracle import build as _build
            _build.build()
        L = ctypes.CDLL(_LIB_PATH)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.oracle_philox4x32_10.restype = None
        L.oracle_thresholds.argtypes = [ctypes.c_double, ctypes.c_double, u32p, u32p,
                                        ctypes.POINTER(ctypes.c_int32)]
        L.oracle_init.argtypes = [ctypes.POINTER(Desc), ctypes.c_void_p]
        L.oracle_observables.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int64)]
        L.oracle_observables.restype = None
        L.oracle_sweeps.argtypes = [ctypes.POINTER(Desc), ctypes.c_void_p, ctypes.c_uint64,
                                    ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p,
                                    ctypes.c_void_p]
        L.oracle_run_batch.argtypes = [ctypes.c_int32, ctypes.POINTER(Desc),
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p,
                                       ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_int32]
        L.oracle_sweeps_rows.argtypes = [ctypes.POINTER(Desc), ctypes.c_void_p, ctypes.c_uint64,
                                         ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_int32]
        L.oracle_bond_threshold.argtypes = [ctypes.c_double, ctypes.c_double, u32p,
                                            ctypes.POINTER(ctypes.c_int32)]
        L.oracle_cluster_labels.argtypes = [ctypes.POINTER(Desc), ctypes.c_void_p, ctypes.c_uint32,
                                            ctypes.c_void_p]
        L.oracle_wolff_seed.argtypes = [ctypes.POINTER(Desc), ctypes.c_uint32]
        L.oracle_wolff_seed.restype = ctypes.c_uint32
        L.oracle_cluster_steps.argtypes = [ctypes.POINTER(Desc), ctypes.c_void_p, ctypes.c_int32,
                                           ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                           ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_run_cluster_batch.argtypes = [ctypes.c_int32, ctypes.POINTER(Desc),
                                               ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                               ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
        L.oracle3_thresholds.argtypes = [ctypes.c_double, ctypes.c_double, u32p, ctypes.POINTER(ctypes.c_int32)]
        L.oracle3_init.argtypes = [ctypes.POINTER(Desc3), ctypes.c_void_p]
        L.oracle3_observables.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.oracle3_observables.restype = None
        L.oracle3_sweeps.argtypes = [ctypes.POINTER(Desc3), ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                     ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
        L.oracle3_run_batch.argtypes = [ctypes.c_int32, ctypes.POINTER(Desc3), ctypes.POINTER(ctypes.c_void_p),
                                        ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_int32]
        _lib = L
    return _lib


def default_threads():
    """Host threads for batched oracle runs: the CPUs this process may use, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


RNG_SITE, RNG_BITSLICED = 0, 1


def desc(Lx, Ly, J=1.0, beta=1.0, seed=0, replica=0, init=INIT_RANDOM, rng=RNG_SITE):
    """rng: RNG_SITE (one Philox word per site) or RNG_BITSLICED (each site's
    uniform is bit b of the 32 words of its 32-site group, transposed)."""
    return Desc(int(Lx), int(Ly), float(J), float(beta), int(seed), int(replica), int(init), int(rng))


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xffffffff for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xffffffff for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().oracle_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def thresholds(J, beta):
    """(thr4, thr8, always) for the Metropolis rule; raises ValueError if invalid."""
    a, b, c = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_int32()
    st = lib().oracle_thresholds(float(J), float(beta), ctypes.byref(a), ctypes.byref(b),
                                 ctypes.byref(c))
    if st != 0:
        raise ValueError("invalid J/beta")
    return int(a.value), int(b.value), int(c.value)


def init_state(d):
    """Initial state of one replica as an (Ly, Lx) int8 array of +-1."""
    s = np.empty((d.Ly, d.Lx), dtype=np.int8)
    st = lib().oracle_init(ctypes.byref(d), s.ctypes.data)
    if st != 0:
        raise ValueError("invalid descriptor")
    return s


def observables(s):
    """(B, M) of an (Ly, Lx) +-1 array: bond sum (E = -J B) and magnetisation."""
    s = np.ascontiguousarray(s, dtype=np.int8)
    B, M = ctypes.c_int64(), ctypes.c_int64()
    lib().oracle_observables(s.shape[1], s.shape[0], s.ctypes.data, ctypes.byref(B),
                             ctypes.byref(M))
    return int(B.value), int(M.value)


def sweeps(d, s, n, t0=0, record_every=0):
    """Run n sweeps in place on s (int8, C-contiguous); returns (bond, mag) traces."""
    assert s.dtype == np.int8 and s.flags.c_contiguous and s.shape == (d.Ly, d.Lx)
    n_rec = n // record_every if record_every else 0
    bond = np.zeros(max(n_rec, 1), dtype=np.int64)
    mag = np.zeros(max(n_rec, 1), dtype=np.int64)
    st = lib().oracle_sweeps(ctypes.byref(d), s.ctypes.data, int(t0), int(n), int(record_every),
                             bond.ctypes.data if n_rec else None,
                             mag.ctypes.data if n_rec else None)
    if st != 0:
        raise ValueError("invalid arguments")
    return bond[:n_rec], mag[:n_rec]


def sweeps_rows(d, s, n, t0=0, record_every=0, threads=None):
    """sweeps() on host threads that split the rows of each colour phase
    (the same result for every thread count)."""
    assert s.dtype == np.int8 and s.flags.c_contiguous and s.shape == (d.Ly, d.Lx)
    n_rec = n // record_every if record_every else 0
    bond = np.zeros(max(n_rec, 1), dtype=np.int64)
    mag = np.zeros(max(n_rec, 1), dtype=np.int64)
    if threads is None:
        threads = default_threads()
    st = lib().oracle_sweeps_rows(ctypes.byref(d), s.ctypes.data, int(t0), int(n), int(record_every),
                                  bond.ctypes.data if n_rec else None,
                                  mag.ctypes.data if n_rec else None, int(threads))
    if st != 0:
        raise ValueError("invalid arguments")
    return bond[:n_rec], mag[:n_rec]


def run_batch(descs, states, n, t0=None, record_every=0, threads=None):
    """Sweep many replicas in place on host threads.

    ``states`` is a list of (Ly, Lx) int8 arrays; returns (bond, mag) traces of
    shape (n_replicas, n // record_every).  A replica larger than an even
    share of the batch (total spins / threads), or any replica when there are
    fewer replicas than threads, runs alone on all threads split over its rows
    (sweeps_rows); the rest run one replica per thread.  Every split gives the
    same result.
    """
    nrep = len(descs)
    for r, s in enumerate(states):
        assert s.dtype == np.int8 and s.flags.c_contiguous
        assert s.shape == (descs[r].Ly, descs[r].Lx)
    n_rec = n // record_every if record_every else 0
    bond = np.zeros((nrep, max(n_rec, 1)), dtype=np.int64)
    mag = np.zeros((nrep, max(n_rec, 1)), dtype=np.int64)
    t0s = np.broadcast_to(np.asarray(0 if t0 is None else t0, dtype=np.uint64), (nrep,))
    if threads is None:
        threads = default_threads()
    sizes = [d.Lx * d.Ly for d in descs]
    share = sum(sizes) / max(threads, 1)
    alone = [r for r in range(nrep) if threads > 1 and (nrep < threads or sizes[r] > share)]
    for r in alone:
        b, m = sweeps_rows(descs[r], states[r], n, int(t0s[r]), record_every, threads)
        bond[r, :n_rec], mag[r, :n_rec] = b, m
    taken = set(alone)
    rest = [r for r in range(nrep) if r not in taken]
    if rest:
        k = len(rest)
        arr = (Desc * k)(*[descs[r] for r in rest])
        ptrs = (ctypes.c_void_p * k)(*[states[r].ctypes.data for r in rest])
        t0a = np.ascontiguousarray(t0s[rest])
        rb = np.zeros((k, max(n_rec, 1)), dtype=np.int64)
        rm = np.zeros((k, max(n_rec, 1)), dtype=np.int64)
        st = lib().oracle_run_batch(k, arr, ptrs, t0a.ctypes.data, int(n), int(record_every),
                                    rb.ctypes.data if n_rec else None,
                                    rm.ctypes.data if n_rec else None, int(threads))
        if st != 0:
            raise ValueError("invalid arguments")
        bond[rest], mag[rest] = rb, rm
    return bond[:, :n_rec], mag[:, :n_rec]


SWENDSEN_WANG, WOLFF = 0, 1


def bond_threshold(J, beta):
    """(thr, none): a bond between aligned spins is occupied iff its word >= thr
    (P = 1 - thr / 2^32, the Fortuin-Kasteleyn 1 - exp(-2 beta J)); none = 1
    when beta * J == 0 (no bond is occupied)."""
    a, c = ctypes.c_uint32(), ctypes.c_int32()
    if lib().oracle_bond_threshold(float(J), float(beta), ctypes.byref(a), ctypes.byref(c)) != 0:
        raise ValueError("invalid J/beta")
    return int(a.value), int(c.value)


def cluster_labels(d, s, t):
    """Cluster roots (smallest site index of each cluster) of the bond
    configuration of step t, as an (Ly, Lx) uint32 array."""
    s = np.ascontiguousarray(s, dtype=np.int8)
    assert s.shape == (d.Ly, d.Lx)
    out = np.empty((d.Ly, d.Lx), dtype=np.uint32)
    if lib().oracle_cluster_labels(ctypes.byref(d), s.ctypes.data, int(t), out.ctypes.data) != 0:
        raise ValueError("invalid arguments")
    return out


def wolff_seed(d, t):
    """Seed site index of the Wolff step with counter t."""
    return int(lib().oracle_wolff_seed(ctypes.byref(d), int(t)))


def cluster_steps(d, s, n, algorithm=SWENDSEN_WANG, t0=0, record_every=0):
    """n cluster steps in place on s (int8, C-contiguous); returns (bond, mag) traces."""
    assert s.dtype == np.int8 and s.flags.c_contiguous and s.shape == (d.Ly, d.Lx)
    n_rec = n // record_every if record_every else 0
    bond = np.zeros(max(n_rec, 1), dtype=np.int64)
    mag = np.zeros(max(n_rec, 1), dtype=np.int64)
    st = lib().oracle_cluster_steps(ctypes.byref(d), s.ctypes.data, int(algorithm), int(t0), int(n),
                                    int(record_every), bond.ctypes.data if n_rec else None,
                                    mag.ctypes.data if n_rec else None)
    if st != 0:
        raise ValueError("invalid arguments")
    return bond[:n_rec], mag[:n_rec]


def run_cluster_batch(descs, states, n, algorithm=SWENDSEN_WANG, t0=None, record_every=0, threads=None):
    """Cluster steps of many replicas in place on host threads (as run_batch)."""
    nrep = len(descs)
    arr = (Desc * nrep)(*descs)
    ptrs = (ctypes.c_void_p * nrep)()
    for r, s in enumerate(states):
        assert s.dtype == np.int8 and s.flags.c_contiguous
        assert s.shape == (descs[r].Ly, descs[r].Lx)
        ptrs[r] = s.ctypes.data
    n_rec = n // record_every if record_every else 0
    bond = np.zeros((nrep, max(n_rec, 1)), dtype=np.int64)
    mag = np.zeros((nrep, max(n_rec, 1)), dtype=np.int64)
    t0a = None
    if t0 is not None:
        t0a = np.ascontiguousarray(np.broadcast_to(np.asarray(t0, dtype=np.uint64), (nrep,)))
    if threads is None:
        threads = default_threads()
    st = lib().oracle_run_cluster_batch(nrep, arr, ptrs, int(algorithm),
                                        t0a.ctypes.data if t0a is not None else None, int(n),
                                        int(record_every), bond.ctypes.data if n_rec else None,
                                        mag.ctypes.data if n_rec else None, int(threads))
    if st != 0:
        raise ValueError("invalid arguments")
    return bond[:, :n_rec], mag[:, :n_rec]


# ---- 3D (simple cubic, six neighbours) ---------------------------------------

def desc3(Lx, Ly, Lz, J=1.0, beta=1.0, seed=0, replica=0, init=INIT_RANDOM, rng=RNG_SITE):
    """rng: RNG_SITE or RNG_BITSLICED, as for desc()."""
    return Desc3(int(Lx), int(Ly), int(Lz), int(init), float(J), float(beta), int(seed), int(replica), int(rng))


def thresholds3(J, beta):
    """(thr4, thr8, thr12, always) of the 3D Metropolis rule."""
    thr = (ctypes.c_uint32 * 3)()
    a = ctypes.c_int32()
    if lib().oracle3_thresholds(float(J), float(beta), thr, ctypes.byref(a)) != 0:
        raise ValueError("invalid J/beta")
    return int(thr[0]), int(thr[1]), int(thr[2]), int(a.value)


def init_state3(d):
    """Initial state of a 3D replica as an (Lz, Ly, Lx) int8 array of +-1."""
    s = np.empty((d.Lz, d.Ly, d.Lx), dtype=np.int8)
    if lib().oracle3_init(ctypes.byref(d), s.ctypes.data) != 0:
        raise ValueError("invalid descriptor")
    return s


def observables3(s):
    """(B, M) of an (Lz, Ly, Lx) +-1 array."""
    s = np.ascontiguousarray(s, dtype=np.int8)
    B, M = ctypes.c_int64(), ctypes.c_int64()
    lib().oracle3_observables(s.shape[2], s.shape[1], s.shape[0], s.ctypes.data, ctypes.byref(B), ctypes.byref(M))
    return int(B.value), int(M.value)


def sweeps3(d, s, n, t0=0, record_every=0):
    """n 3D sweeps in place on s; returns (bond, mag) traces."""
    assert s.dtype == np.int8 and s.flags.c_contiguous and s.shape == (d.Lz, d.Ly, d.Lx)
    n_rec = n // record_every if record_every else 0
    bond = np.zeros(max(n_rec, 1), dtype=np.int64)
    mag = np.zeros(max(n_rec, 1), dtype=np.int64)
    if lib().oracle3_sweeps(ctypes.byref(d), s.ctypes.data, int(t0), int(n), int(record_every),
                            bond.ctypes.data if n_rec else None, mag.ctypes.data if n_rec else None) != 0:
        raise ValueError("invalid arguments")
    return bond[:n_rec], mag[:n_rec]


def run_batch3(descs, states, n, t0=None, record_every=0, threads=None):
    """3D sweeps of many replicas in place on host threads (as run_batch)."""
    nrep = len(descs)
    arr = (Desc3 * nrep)(*descs)
    ptrs = (ctypes.c_void_p * nrep)()
    for r, s in enumerate(states):
        assert s.dtype == np.int8 and s.flags.c_contiguous and s.shape == (descs[r].Lz, descs[r].Ly, descs[r].Lx)
        ptrs[r] = s.ctypes.data
    n_rec = n // record_every if record_every else 0
    bond = np.zeros((nrep, max(n_rec, 1)), dtype=np.int64)
    mag = np.zeros((nrep, max(n_rec, 1)), dtype=np.int64)
    t0a = None
    if t0 is not None:
        t0a = np.ascontiguousarray(np.broadcast_to(np.asarray(t0, dtype=np.uint64), (nrep,)))
    if threads is None:
        threads = default_threads()
    if lib().oracle3_run_batch(nrep, arr, ptrs, t0a.ctypes.data if t0a is not None else None, int(n),
                               int(record_every), bond.ctypes.data if n_rec else None,
                               mag.ctypes.data if n_rec else None, int(threads)) != 0:
        raise ValueError("invalid arguments")
    return bond[:, :n_rec], mag[:, :n_rec]
