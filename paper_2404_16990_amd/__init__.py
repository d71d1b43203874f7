"""Python binding of libising.so, the MI355X checkerboard Metropolis library.

Argument marshalling only: every step of a sweep runs in the library's HIP
kernels.  The functions keep the C ABI's names (see include/ising.h);
``Batch`` is a convenience owner of the device buffer (a torch uint8 tensor)
that calls them.  Importing works without a GPU; calls that touch the device
need one.  There is no fallback: if the library is missing, every call raises.
"""
import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_lib", "libising.so")

ISING_OK = 0
ISING_E_INVALID = -1
ISING_E_UNSUPPORTED = -2
ISING_E_NOMEM = -3
ISING_E_HIP = -4
ISING_E_STATE = -5
ISING_INIT_RANDOM, ISING_INIT_UP, ISING_INIT_DOWN = 0, 1, 2

EXPORTED = [
    "ising_strerror", "ising_last_error", "ising_state_bytes", "ising_batch_create",
    "ising_batch_run", "ising_batch_observables", "ising_batch_get_spins",
    "ising_batch_set_spins", "ising_batch_get_sweep", "ising_batch_set_sweep",
    "ising_batch_set_beta", "ising_batch_get_schedule", "ising_batch_set_schedule",
    "ising_batch_mode_counts", "ising_batch_graph_stats", "ising_batch_autotune", "ising_batch_destroy",
    "ising_nn_param_count", "ising_nn_state_bytes", "ising_nn_create", "ising_nn_get_params",
    "ising_nn_set_params", "ising_nn_forward_backward", "ising_nn_train_step", "ising_nn_train_step_sampled",
    "ising_nn_train_steps_sampled", "ising_nn_score",
    "ising_nn_sample", "ising_batch_extract_blocks", "ising_batch_block_round", "ising_nn_graph_stats",
    "ising_nn_destroy",
    "ising_cluster_ws_bytes", "ising_batch_cluster", "ising_batch_cluster_static",
    "ising3d_state_bytes", "ising3d_batch_create", "ising3d_batch_run", "ising3d_batch_observables",
    "ising3d_batch_get_spins", "ising3d_batch_set_spins", "ising3d_batch_get_sweep", "ising3d_batch_destroy",
]


class ising_desc(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32), ("J", ctypes.c_double),
                ("beta", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("replica", ctypes.c_uint32), ("init", ctypes.c_int32), ("rng", ctypes.c_int32)]


ISING_RNG_SITE, ISING_RNG_BITSLICED = 0, 1
ISING_CLUSTER_SWENDSEN_WANG, ISING_CLUSTER_WOLFF = 0, 1


class ising3d_desc(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32), ("Lz", ctypes.c_int32), ("init", ctypes.c_int32),
                ("J", ctypes.c_double), ("beta", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("replica", ctypes.c_uint32), ("rng", ctypes.c_int32)]


class ising_schedule(ctypes.Structure):
    _fields_ = [("word_bits", ctypes.c_int32), ("resident_max_bytes", ctypes.c_int32),
                ("resident_threads", ctypes.c_int32), ("stream_threads", ctypes.c_int32),
                ("stream_words", ctypes.c_int32), ("sweeps_per_launch", ctypes.c_int32),
                ("use_graph", ctypes.c_int32)]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class IsingError(RuntimeError):
    def __init__(self, code, func, detail):
        self.code = code
        super().__init__(f"{func} failed ({code}: {detail})")


_lib = None


def lib():
    """Load libising.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2404_16990_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
        P = ctypes.POINTER
        L.ising_strerror.argtypes = [ctypes.c_int]
        L.ising_strerror.restype = ctypes.c_char_p
        L.ising_last_error.argtypes = []
        L.ising_last_error.restype = ctypes.c_char_p
        L.ising_state_bytes.argtypes = [i32, P(ising_desc), P(ctypes.c_size_t)]
        L.ising_batch_create.argtypes = [i32, P(ising_desc), vp, ctypes.c_size_t, vp, P(vp)]
        L.ising_batch_run.argtypes = [vp, u64, u32, vp, vp, vp]
        L.ising_batch_observables.argtypes = [vp, vp, vp, vp]
        L.ising_batch_get_spins.argtypes = [vp, i32, vp, vp]
        L.ising_batch_set_spins.argtypes = [vp, i32, vp, vp]
        L.ising_batch_get_sweep.argtypes = [vp, i32, P(u64), vp]
        L.ising_batch_set_sweep.argtypes = [vp, i32, u64, vp]
        L.ising_batch_set_beta.argtypes = [vp, i32, ctypes.c_double, vp]
        L.ising_batch_get_schedule.argtypes = [vp, P(ising_schedule)]
        L.ising_batch_set_schedule.argtypes = [vp, P(ising_schedule)]
        L.ising_batch_mode_counts.argtypes = [vp, P(i32), P(i32)]
        L.ising_batch_graph_stats.argtypes = [vp, P(i32), P(ctypes.c_int64)]
        L.ising_batch_autotune.argtypes = [vp, i32, P(ising_schedule), P(i32), vp]
        L.ising_batch_destroy.argtypes = [vp]
        f32 = ctypes.c_float
        L.ising_nn_param_count.argtypes = [i32, P(i32)]
        L.ising_nn_state_bytes.argtypes = [i32, i32, i32, i32, P(ctypes.c_size_t)]
        L.ising_nn_create.argtypes = [i32, i32, i32, i32, vp, vp, ctypes.c_size_t, vp, P(vp)]
        L.ising_nn_get_params.argtypes = [vp, vp, vp]
        L.ising_nn_set_params.argtypes = [vp, vp, vp]
        L.ising_nn_forward_backward.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, vp]
        L.ising_nn_train_step.argtypes = [vp, vp, vp, vp, i32, f32, vp, vp]
        L.ising_nn_train_step_sampled.argtypes = [vp, vp, vp, vp, ctypes.c_int64, i32, f32, u64, vp, vp]
        L.ising_nn_train_steps_sampled.argtypes = [vp, vp, vp, vp, ctypes.c_int64, i32, f32, u64, ctypes.c_int64,
                                                   vp, vp]
        L.ising_nn_score.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        L.ising_nn_sample.argtypes = [vp, i32, vp, vp, u64, u32, u32, u32, vp, vp, vp]
        L.ising_batch_extract_blocks.argtypes = [vp, i32, i32, u32, vp, vp, vp, vp]
        L.ising_batch_block_round.argtypes = [vp, vp, u32, vp, vp]
        L.ising_nn_graph_stats.argtypes = [vp, P(i32), P(ctypes.c_int64)]
        L.ising_nn_destroy.argtypes = [vp]
        L.ising_cluster_ws_bytes.argtypes = [vp, P(ctypes.c_size_t)]
        L.ising_batch_cluster.argtypes = [vp, i32, u64, u32, vp, ctypes.c_size_t, vp, vp, vp]
        L.ising_batch_cluster_static.argtypes = [vp, i32, u64, u32, vp, vp, vp]
        L.ising3d_state_bytes.argtypes = [i32, P(ising3d_desc), P(ctypes.c_size_t)]
        L.ising3d_batch_create.argtypes = [i32, P(ising3d_desc), vp, ctypes.c_size_t, vp, P(vp)]
        L.ising3d_batch_run.argtypes = [vp, u64, u32, vp, vp, vp]
        L.ising3d_batch_observables.argtypes = [vp, vp, vp, vp]
        L.ising3d_batch_get_spins.argtypes = [vp, i32, vp, vp]
        L.ising3d_batch_set_spins.argtypes = [vp, i32, vp, vp]
        L.ising3d_batch_get_sweep.argtypes = [vp, i32, P(u64), vp]
        L.ising3d_batch_destroy.argtypes = [vp]
        for name in EXPORTED[2:]:
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(code, func):
    if code != ISING_OK:
        detail = lib().ising_last_error().decode() or lib().ising_strerror(code).decode()
        raise IsingError(code, func, detail)


def _descs(descs):
    arr = (ising_desc * len(descs))()
    for i, d in enumerate(descs):
        if isinstance(d, ising_desc):
            arr[i] = d
        else:
            arr[i] = ising_desc(int(d["Lx"]), int(d["Ly"]), float(d.get("J", 1.0)), float(d["beta"]),
                                int(d["seed"]), int(d["replica"]), int(d.get("init", 0)), int(d.get("rng", 0)))
    return arr


# ---- same names as the C ABI ------------------------------------------------

def ising_strerror(code):
    return lib().ising_strerror(int(code)).decode()


def ising_last_error():
    return lib().ising_last_error().decode()


def ising_state_bytes(descs):
    arr = _descs(descs)
    n = ctypes.c_size_t()
    _check(lib().ising_state_bytes(len(arr), arr, ctypes.byref(n)), "ising_state_bytes")
    return int(n.value)


def ising_batch_create(descs, dev_buf, nbytes, stream=None):
    arr = _descs(descs)
    h = ctypes.c_void_p()
    _check(lib().ising_batch_create(len(arr), arr, dev_buf, nbytes, stream, ctypes.byref(h)),
           "ising_batch_create")
    return h


def ising_batch_run(h, n_sweeps, record_every=0, dev_bond=None, dev_mag=None, stream=None):
    _check(lib().ising_batch_run(h, int(n_sweeps), int(record_every), dev_bond, dev_mag, stream),
           "ising_batch_run")


def ising_batch_observables(h, host_bond, host_mag, stream=None):
    _check(lib().ising_batch_observables(h, host_bond, host_mag, stream), "ising_batch_observables")


def ising_batch_get_spins(h, r, host_pm1, stream=None):
    _check(lib().ising_batch_get_spins(h, int(r), host_pm1, stream), "ising_batch_get_spins")


def ising_batch_set_spins(h, r, host_pm1, stream=None):
    _check(lib().ising_batch_set_spins(h, int(r), host_pm1, stream), "ising_batch_set_spins")


def ising_batch_get_sweep(h, r, stream=None):
    t = ctypes.c_uint64()
    _check(lib().ising_batch_get_sweep(h, int(r), ctypes.byref(t), stream), "ising_batch_get_sweep")
    return int(t.value)


def ising_batch_set_sweep(h, r, t, stream=None):
    _check(lib().ising_batch_set_sweep(h, int(r), int(t), stream), "ising_batch_set_sweep")


def ising_batch_set_beta(h, r, beta, stream=None):
    _check(lib().ising_batch_set_beta(h, int(r), float(beta), stream), "ising_batch_set_beta")


def ising_batch_get_schedule(h):
    s = ising_schedule()
    _check(lib().ising_batch_get_schedule(h, ctypes.byref(s)), "ising_batch_get_schedule")
    return s


def ising_batch_set_schedule(h, sched):
    if isinstance(sched, dict):
        s = ising_schedule(**{k: int(v) for k, v in sched.items()})
    else:
        s = sched
    _check(lib().ising_batch_set_schedule(h, ctypes.byref(s)), "ising_batch_set_schedule")


def ising_batch_mode_counts(h):
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().ising_batch_mode_counts(h, ctypes.byref(a), ctypes.byref(b)), "ising_batch_mode_counts")
    return int(a.value), int(b.value)


def ising_batch_graph_stats(h):
    """Returns (executable graphs held now, captures since creation)."""
    a, b = ctypes.c_int32(), ctypes.c_int64()
    _check(lib().ising_batch_graph_stats(h, ctypes.byref(a), ctypes.byref(b)), "ising_batch_graph_stats")
    return int(a.value), int(b.value)


def ising_batch_autotune(h, trial_sweeps, stream=None):
    """Returns (installed schedule, number of candidates timed; 0 on a cache hit)."""
    s = ising_schedule()
    n = ctypes.c_int32()
    _check(lib().ising_batch_autotune(h, int(trial_sweeps), ctypes.byref(s), ctypes.byref(n), stream),
           "ising_batch_autotune")
    return s, int(n.value)


def ising_batch_destroy(h):
    _check(lib().ising_batch_destroy(h), "ising_batch_destroy")


def _descs3(descs):
    arr = (ising3d_desc * len(descs))()
    for i, d in enumerate(descs):
        if isinstance(d, ising3d_desc):
            arr[i] = d
        else:
            arr[i] = ising3d_desc(int(d["Lx"]), int(d["Ly"]), int(d["Lz"]), int(d.get("init", 0)),
                                  float(d.get("J", 1.0)), float(d["beta"]), int(d["seed"]), int(d["replica"]),
                                  int(d.get("rng", 0)))
    return arr


def ising3d_state_bytes(descs):
    out = ctypes.c_size_t()
    _check(lib().ising3d_state_bytes(len(descs), _descs3(descs), ctypes.byref(out)), "ising3d_state_bytes")
    return int(out.value)


def ising3d_batch_create(descs, dev_buf, nbytes, stream=None):
    h = ctypes.c_void_p()
    _check(lib().ising3d_batch_create(len(descs), _descs3(descs), dev_buf, nbytes, stream, ctypes.byref(h)),
           "ising3d_batch_create")
    return h


def ising3d_batch_run(h, n_sweeps, record_every=0, dev_bond=None, dev_mag=None, stream=None):
    _check(lib().ising3d_batch_run(h, n_sweeps, record_every, dev_bond, dev_mag, stream), "ising3d_batch_run")


def ising3d_batch_observables(h, host_bond, host_mag, stream=None):
    _check(lib().ising3d_batch_observables(h, host_bond, host_mag, stream), "ising3d_batch_observables")


def ising3d_batch_get_spins(h, r, host_pm1, stream=None):
    _check(lib().ising3d_batch_get_spins(h, r, host_pm1, stream), "ising3d_batch_get_spins")


def ising3d_batch_set_spins(h, r, host_pm1, stream=None):
    _check(lib().ising3d_batch_set_spins(h, r, host_pm1, stream), "ising3d_batch_set_spins")


def ising3d_batch_get_sweep(h, r, stream=None):
    t = ctypes.c_uint64()
    _check(lib().ising3d_batch_get_sweep(h, r, ctypes.byref(t), stream), "ising3d_batch_get_sweep")
    return int(t.value)


def ising3d_batch_destroy(h):
    _check(lib().ising3d_batch_destroy(h), "ising3d_batch_destroy")


def ising_cluster_ws_bytes(h):
    out = ctypes.c_size_t()
    _check(lib().ising_cluster_ws_bytes(h, ctypes.byref(out)), "ising_cluster_ws_bytes")
    return int(out.value)


def ising_batch_cluster(h, algorithm, n_steps, record_every, dev_ws, ws_bytes, dev_bond=None, dev_mag=None,
                        stream=None):
    _check(lib().ising_batch_cluster(h, algorithm, n_steps, record_every, dev_ws, ws_bytes, dev_bond, dev_mag,
                                     stream), "ising_batch_cluster")


ISING_CLUSTER_STATIC_WS_BYTES = 64 << 20


def ising_batch_cluster_static(h, algorithm, n_steps, record_every, dev_bond=None, dev_mag=None, stream=None):
    _check(lib().ising_batch_cluster_static(h, algorithm, n_steps, record_every, dev_bond, dev_mag, stream),
           "ising_batch_cluster_static")


def ising_nn_param_count(channels=64):
    n = ctypes.c_int32()
    _check(lib().ising_nn_param_count(int(channels), ctypes.byref(n)), "ising_nn_param_count")
    return int(n.value)


def ising_nn_state_bytes(block, channels, max_batch, max_seq):
    n = ctypes.c_size_t()
    _check(lib().ising_nn_state_bytes(int(block), int(channels), int(max_batch), int(max_seq), ctypes.byref(n)),
           "ising_nn_state_bytes")
    return int(n.value)


def ising_nn_create(block, channels, max_batch, max_seq, host_params, dev_buf, nbytes, stream=None):
    h = ctypes.c_void_p()
    _check(lib().ising_nn_create(int(block), int(channels), int(max_batch), int(max_seq), host_params, dev_buf,
                                 nbytes, stream, ctypes.byref(h)), "ising_nn_create")
    return h


def ising_nn_get_params(m, host_params, stream=None):
    _check(lib().ising_nn_get_params(m, host_params, stream), "ising_nn_get_params")


def ising_nn_set_params(m, host_params, stream=None):
    _check(lib().ising_nn_set_params(m, host_params, stream), "ising_nn_set_params")


def ising_nn_forward_backward(m, blocks, bnd, coupling, batch, logits, grad, loss, stream=None):
    _check(lib().ising_nn_forward_backward(m, blocks, bnd, coupling, int(batch), logits, grad, loss, stream),
           "ising_nn_forward_backward")


def ising_nn_train_step(m, blocks, bnd, coupling, batch, lr, loss, stream=None):
    _check(lib().ising_nn_train_step(m, blocks, bnd, coupling, int(batch), float(lr), loss, stream),
           "ising_nn_train_step")


def ising_nn_train_step_sampled(m, blocks, bnd, coupling, n_rows, batch, lr, seed, loss, stream=None):
    _check(lib().ising_nn_train_step_sampled(m, blocks, bnd, coupling, int(n_rows), int(batch), float(lr),
                                             int(seed), loss, stream), "ising_nn_train_step_sampled")


def ising_nn_train_steps_sampled(m, blocks, bnd, coupling, n_rows, batch, lr, seed, n_steps, loss, stream=None):
    _check(lib().ising_nn_train_steps_sampled(m, blocks, bnd, coupling, int(n_rows), int(batch), float(lr),
                                              int(seed), int(n_steps), loss, stream),
           "ising_nn_train_steps_sampled")


def ising_nn_score(m, n, blocks, bnd, coupling, logq, stream=None):
    _check(lib().ising_nn_score(m, int(n), blocks, bnd, coupling, logq, stream), "ising_nn_score")


def ising_nn_sample(m, n, bnd, coupling, seed, replica, round_, blk0, blocks_out, logq, stream=None):
    _check(lib().ising_nn_sample(m, int(n), bnd, coupling, int(seed), int(replica), int(round_), int(blk0),
                                 blocks_out, logq, stream), "ising_nn_sample")


def ising_batch_extract_blocks(b, block, per_replica, draw, blocks, bnd, coupling, stream=None):
    _check(lib().ising_batch_extract_blocks(b, int(block), int(per_replica), int(draw), blocks, bnd, coupling,
                                            stream), "ising_batch_extract_blocks")


def ising_batch_block_round(b, m, round_, accepts=None, stream=None):
    _check(lib().ising_batch_block_round(b, m, int(round_), accepts, stream), "ising_batch_block_round")


def ising_nn_graph_stats(m):
    n = ctypes.c_int32()
    c = ctypes.c_int64()
    _check(lib().ising_nn_graph_stats(m, ctypes.byref(n), ctypes.byref(c)), "ising_nn_graph_stats")
    return int(n.value), int(c.value)


def ising_nn_destroy(m):
    _check(lib().ising_nn_destroy(m), "ising_nn_destroy")


# ---- convenience owner -------------------------------------------------------

class Batch:
    """A batch of replicas in a torch-owned device buffer on the current device."""

    def __init__(self, descs, stream=None, device="cuda"):
        import torch
        self.torch = torch
        self.descs = list(descs)
        self.n = len(self.descs)
        self.nbytes = ising_state_bytes(self.descs)
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.buf.device)
        self.h = ising_batch_create(self.descs, self.buf.data_ptr(), self.nbytes, self._s())

    def _s(self):
        return ctypes.c_void_p(self.stream.cuda_stream)

    def _spins(self, r):
        d = self.descs[r]
        return (d["Ly"], d["Lx"]) if isinstance(d, dict) else (d.Ly, d.Lx)

    def run(self, n_sweeps, record_every=0):
        """Enqueue n_sweeps sweeps; returns device (bond, mag) traces or None."""
        torch = self.torch
        n_rec = n_sweeps // record_every if record_every else 0
        if n_rec:
            bond = torch.empty((self.n, n_rec), dtype=torch.int64, device=self.buf.device)
            mag = torch.empty((self.n, n_rec), dtype=torch.int64, device=self.buf.device)
            ising_batch_run(self.h, n_sweeps, record_every, bond.data_ptr(), mag.data_ptr(), self._s())
            return bond, mag
        ising_batch_run(self.h, n_sweeps, 0, None, None, self._s())
        return None

    def cluster(self, n_steps, algorithm="sw", record_every=0):
        """Enqueue n_steps Swendsen-Wang ("sw") or Wolff ("wolff") cluster
        steps; returns device (bond, mag) traces or None.  The workspace is a
        torch buffer kept for later calls."""
        torch = self.torch
        algo = {"sw": ISING_CLUSTER_SWENDSEN_WANG, "wolff": ISING_CLUSTER_WOLFF}[algorithm]
        need = ising_cluster_ws_bytes(self.h)
        if getattr(self, "ws", None) is None or self.ws.numel() < need:
            self.ws = torch.empty(need, dtype=torch.uint8, device=self.buf.device)
        n_rec = n_steps // record_every if record_every else 0
        if n_rec:
            bond = torch.empty((self.n, n_rec), dtype=torch.int64, device=self.buf.device)
            mag = torch.empty((self.n, n_rec), dtype=torch.int64, device=self.buf.device)
            ising_batch_cluster(self.h, algo, n_steps, record_every, self.ws.data_ptr(), self.ws.numel(),
                                bond.data_ptr(), mag.data_ptr(), self._s())
            return bond, mag
        ising_batch_cluster(self.h, algo, n_steps, 0, self.ws.data_ptr(), self.ws.numel(), None, None, self._s())
        return None

    def cluster_static(self, n_steps, algorithm="sw", bond=None, mag=None, record_every=0):
        """cluster() on the library's own workspace (ising_batch_cluster_static):
        the call allocates nothing; traces, if wanted, are caller tensors of
        shape (n, n_steps // record_every), int64."""
        algo = {"sw": ISING_CLUSTER_SWENDSEN_WANG, "wolff": ISING_CLUSTER_WOLFF}[algorithm]
        if record_every:
            n_rec = n_steps // record_every
            for t in (bond, mag):
                if t is None or tuple(t.shape) != (self.n, n_rec) or t.dtype != self.torch.int64 \
                        or not t.is_contiguous():
                    raise ValueError("bond and mag must be contiguous int64 tensors of shape (n, n_steps // every)")
            ising_batch_cluster_static(self.h, algo, n_steps, record_every, bond.data_ptr(), mag.data_ptr(),
                                       self._s())
        else:
            ising_batch_cluster_static(self.h, algo, n_steps, 0, None, None, self._s())

    def observables(self):
        import numpy as np
        b = np.zeros(self.n, dtype=np.int64)
        m = np.zeros(self.n, dtype=np.int64)
        ising_batch_observables(self.h, b.ctypes.data, m.ctypes.data, self._s())
        return b, m

    def get_spins(self, r):
        import numpy as np
        out = np.empty(self._spins(r), dtype=np.int8)
        ising_batch_get_spins(self.h, r, out.ctypes.data, self._s())
        return out

    def set_spins(self, r, s):
        import numpy as np
        s = np.ascontiguousarray(s, dtype=np.int8)
        assert s.shape == self._spins(r)
        ising_batch_set_spins(self.h, r, s.ctypes.data, self._s())

    def get_sweep(self, r):
        return ising_batch_get_sweep(self.h, r, self._s())

    def set_sweep(self, r, t):
        ising_batch_set_sweep(self.h, r, t, self._s())

    def set_beta(self, r, beta):
        ising_batch_set_beta(self.h, r, beta, self._s())

    @property
    def schedule(self):
        return ising_batch_get_schedule(self.h).as_dict()

    def set_schedule(self, **kw):
        s = self.schedule
        s.update(kw)
        ising_batch_set_schedule(self.h, s)

    def mode_counts(self):
        return ising_batch_mode_counts(self.h)

    def graph_stats(self):
        return ising_batch_graph_stats(self.h)

    def autotune(self, trial_sweeps=10):
        s, n = ising_batch_autotune(self.h, trial_sweeps, self._s())
        return s.as_dict(), n

    def close(self):
        if getattr(self, "h", None) is not None:
            ising_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Net:
    """A block-proposal network in a torch-owned device buffer (see include/ising.h)."""

    def __init__(self, params, block=8, max_batch=512, max_seq=65536, stream=None, device="cuda"):
        import numpy as np
        import torch
        self.torch = torch
        self.block = int(block)
        self.max_batch, self.max_seq = int(max_batch), int(max_seq)
        self.n_params = ising_nn_param_count(64)
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.shape == (self.n_params,)
        self.nbytes = ising_nn_state_bytes(self.block, 64, self.max_batch, self.max_seq)
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.buf.device)
        self.h = ising_nn_create(self.block, 64, self.max_batch, self.max_seq, p.ctypes.data, self.buf.data_ptr(),
                                 self.nbytes, self._s())

    def _s(self):
        return ctypes.c_void_p(self.stream.cuda_stream)

    @property
    def params(self):
        import numpy as np
        out = np.empty(self.n_params, dtype=np.float32)
        ising_nn_get_params(self.h, out.ctypes.data, self._s())
        return out

    def set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        ising_nn_set_params(self.h, p.ctypes.data, self._s())

    def forward_backward(self, blocks, bnd, coupling):
        """Device tensors in; returns (logits [n, Bs*Bs], grad [n_params], loss) as device tensors."""
        torch = self.torch
        n = blocks.shape[0]
        logits = torch.empty((n, self.block * self.block), dtype=torch.float32, device=blocks.device)
        grad = torch.empty(self.n_params, dtype=torch.float32, device=blocks.device)
        loss = torch.empty(1, dtype=torch.float32, device=blocks.device)
        ising_nn_forward_backward(self.h, blocks.data_ptr(), bnd.data_ptr(), coupling.data_ptr(), n,
                                  logits.data_ptr(), grad.data_ptr(), loss.data_ptr(), self._s())
        return logits, grad, loss

    def train_step(self, blocks, bnd, coupling, lr, loss=None):
        ising_nn_train_step(self.h, blocks.data_ptr(), bnd.data_ptr(), coupling.data_ptr(), blocks.shape[0],
                            lr, loss.data_ptr() if loss is not None else None, self._s())

    def train_step_sampled(self, blocks, bnd, coupling, batch, lr, seed, loss=None):
        """One Adam step on `batch` rows of the training set (blocks, bnd, coupling)
        drawn on the device from the Philox stream of `seed` and the step count."""
        ising_nn_train_step_sampled(self.h, blocks.data_ptr(), bnd.data_ptr(), coupling.data_ptr(),
                                    blocks.shape[0], batch, lr, seed,
                                    loss.data_ptr() if loss is not None else None, self._s())

    def train_steps_sampled(self, blocks, bnd, coupling, batch, lr, seed, n_steps, loss=None):
        """n_steps consecutive train_step_sampled steps in one call (replays of
        graphs of up to 16 captured steps); loss receives the last step's."""
        ising_nn_train_steps_sampled(self.h, blocks.data_ptr(), bnd.data_ptr(), coupling.data_ptr(),
                                     blocks.shape[0], batch, lr, seed, n_steps,
                                     loss.data_ptr() if loss is not None else None, self._s())

    def score(self, blocks, bnd, coupling):
        torch = self.torch
        n = blocks.shape[0]
        logq = torch.empty(n, dtype=torch.float64, device=blocks.device)
        ising_nn_score(self.h, n, blocks.data_ptr(), bnd.data_ptr(), coupling.data_ptr(), logq.data_ptr(),
                       self._s())
        return logq

    def sample(self, bnd, coupling, seed, replica, round_, blk0=0):
        torch = self.torch
        n = bnd.shape[0]
        out = torch.empty((n, self.block * self.block), dtype=torch.int8, device=bnd.device)
        logq = torch.empty(n, dtype=torch.float64, device=bnd.device)
        ising_nn_sample(self.h, n, bnd.data_ptr(), coupling.data_ptr(), seed, replica, round_, blk0,
                        out.data_ptr(), logq.data_ptr(), self._s())
        return out, logq

    def graph_stats(self):
        """(captured training steps held, captured since creation)."""
        return ising_nn_graph_stats(self.h)

    def close(self):
        if getattr(self, "h", None) is not None:
            ising_nn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _batch_block_round(self, net, round_, accepts=None):
    ising_batch_block_round(self.h, net.h, round_, accepts.data_ptr() if accepts is not None else None, self._s())


def _batch_extract(self, block, per_replica, draw, out=None):
    """Training blocks of every replica; `out` = (blocks, bnd, coupling) views
    with room for n * per_replica rows receive them in place."""
    torch = self.torch
    n = self.n * per_replica
    if out is None:
        blocks = torch.empty((n, block * block), dtype=torch.int8, device=self.buf.device)
        bnd = torch.empty((n, 4 * block), dtype=torch.int8, device=self.buf.device)
        coup = torch.empty(n, dtype=torch.float32, device=self.buf.device)
    else:
        blocks, bnd, coup = out
        if not (blocks.shape == (n, block * block) and bnd.shape == (n, 4 * block) and coup.shape == (n,)
                and blocks.dtype == torch.int8 and bnd.dtype == torch.int8 and coup.dtype == torch.float32
                and blocks.is_contiguous() and bnd.is_contiguous() and coup.is_contiguous()):
            raise ValueError("out views must be contiguous int8 [n, B*B], int8 [n, 4B], float32 [n]")
    ising_batch_extract_blocks(self.h, block, per_replica, draw, blocks.data_ptr(), bnd.data_ptr(),
                               coup.data_ptr(), self._s())
    return blocks, bnd, coup


Batch.block_round = _batch_block_round
Batch.extract_blocks = _batch_extract


class Batch3:
    """A batch of 3D replicas in a torch-owned device buffer on the current device."""

    def __init__(self, descs, stream=None, device="cuda"):
        import torch
        self.torch = torch
        self.descs = list(descs)
        self.n = len(self.descs)
        self.nbytes = ising3d_state_bytes(self.descs)
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.buf.device)
        self.h = ising3d_batch_create(self.descs, self.buf.data_ptr(), self.nbytes, self._s())

    def _s(self):
        return ctypes.c_void_p(self.stream.cuda_stream)

    def _shape(self, r):
        d = self.descs[r]
        return (d["Lz"], d["Ly"], d["Lx"]) if isinstance(d, dict) else (d.Lz, d.Ly, d.Lx)

    def run(self, n_sweeps, record_every=0):
        """Enqueue n_sweeps sweeps; returns device (bond, mag) traces or None."""
        torch = self.torch
        n_rec = n_sweeps // record_every if record_every else 0
        if n_rec:
            bond = torch.empty((self.n, n_rec), dtype=torch.int64, device=self.buf.device)
            mag = torch.empty((self.n, n_rec), dtype=torch.int64, device=self.buf.device)
            ising3d_batch_run(self.h, n_sweeps, record_every, bond.data_ptr(), mag.data_ptr(), self._s())
            return bond, mag
        ising3d_batch_run(self.h, n_sweeps, 0, None, None, self._s())
        return None

    def observables(self):
        import numpy as np
        b = np.zeros(self.n, dtype=np.int64)
        m = np.zeros(self.n, dtype=np.int64)
        ising3d_batch_observables(self.h, b.ctypes.data, m.ctypes.data, self._s())
        return b, m

    def get_spins(self, r):
        import numpy as np
        out = np.empty(self._shape(r), dtype=np.int8)
        ising3d_batch_get_spins(self.h, r, out.ctypes.data, self._s())
        return out

    def set_spins(self, r, s):
        import numpy as np
        s = np.ascontiguousarray(s, dtype=np.int8)
        assert s.shape == self._shape(r)
        ising3d_batch_set_spins(self.h, r, s.ctypes.data, self._s())

    def get_sweep(self, r):
        return ising3d_batch_get_sweep(self.h, r, self._s())

    def close(self):
        if getattr(self, "h", None) is not None:
            ising3d_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
