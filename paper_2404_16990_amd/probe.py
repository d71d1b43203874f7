"""Measured issue costs of the sweep's instructions and HBM copy bandwidth.

Runs the probes in libising_probe.so (built beside libising.so).  The ALU
ceiling of the sweep is 256 CUs x 64 lanes x clock divided by the lane-cycles
one flip attempt needs; the lane-cycle cost of each instruction is measured
here relative to a full-rate 32-bit XOR.  Usage: ``python -m paper_2404_16990_amd.probe``.
"""
import ctypes
import json
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_lib", "libising_probe.so")
NAMES = ["v_mad_u64_u32", "v_mul_hi_u32", "v_mul_lo_u32", "v_bitop3_b32", "v_xor_b32", "v_add_u32",
         "philox4x32_10", "v_lshl_add_u64", "v_addc_co_u32", "v_cmp_lt_u32+v_add_u32", "v_bfe_i32",
         "v_alignbit_b32", "v_cndmask_b32"]
CUS, LANES = 256, 64


def _lib():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} missing: run python -m paper_2404_16990_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    L.ising_probe_alu.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_float)]
    L.ising_probe_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_float)]
    return L


def measure(blocks=256 * 16, iters=4096):
    import torch
    L = _lib()
    out = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    res = {}
    for which, name in enumerate(NAMES):
        ms = ctypes.c_float()
        st = L.ising_probe_alu(which, out.data_ptr(), blocks, iters, ctypes.byref(ms))
        if st != 0:
            raise RuntimeError(f"probe {name} failed ({st})")
        per_thread = iters * (4 if name == "philox4x32_10" else 8)
        res[name] = blocks * 256 * per_thread / (ms.value * 1e-3)
    xor = res["v_xor_b32"]
    lane_clock = xor / (CUS * LANES)  # full-rate ops per lane per second = effective clock
    costs = {k: xor / v for k, v in res.items() if k != "philox4x32_10"}
    return {"ops_per_s": res, "lane_cycles": costs, "effective_clock_hz": lane_clock,
            "philox_calls_per_s": res["philox4x32_10"],
            "philox_lane_cycles_per_call": xor / res["philox4x32_10"]}


def mix_rate(word_bits=64, blocks=256 * 16, iters=128, T=2.269185, rng=0, reps=5, bonds=0):
    """Measured ALU ceiling of the sweep's per-word arithmetic, in site updates
    (flip attempts) per second: k_mix runs ising::update_word on two
    register-resident words per thread (classification, Philox4x32-10,
    acceptance) with no memory traffic and no dependence between updates, in
    the streaming and the LDS-resident kernels' launch shapes; the best of
    `reps` timed launches per shape after a warm-up launch.  bonds=0: random
    neighbour words (half the bonds anti-aligned); bonds=1: about 1/8 of the
    bonds anti-aligned, as in a 2D lattice near T_c (this matters for the
    bit-sliced contract only, whose lazy comparison depends on how many sites
    are undecided)."""
    import math
    import torch
    L = _lib()
    L.ising_probe_mix.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_uint,
                                  ctypes.c_uint, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_float)]
    thr = [min(int(math.floor(math.ldexp(math.exp(-4.0 * k / T), 32))), 2**32 - 1) for k in (1, 2)]
    out = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    ms = ctypes.c_float()
    if L.ising_probe_mix(int(word_bits), out.data_ptr(), blocks, iters, thr[0], thr[1], int(rng), int(bonds),
                         int(reps), ctypes.byref(ms)) != 0:
        raise RuntimeError("mix probe failed")
    return blocks * 256 * iters * 2 * word_bits / (ms.value * 1e-3)


def mix3_rate(blocks=256 * 16, iters=64, T=4.5115, rng=0, bonds=0):
    """Measured ALU ceiling of the 3D sweep's per-word arithmetic (flip
    attempts per second): k_mix3 runs ising::flip_mask32_3d on
    register-resident words with no memory traffic; bonds=1 gives the
    neighbour words the bond statistics of the 3D model near T_c (about a
    third of the bonds anti-aligned) instead of random words."""
    import math
    import torch
    L = _lib()
    L.ising_probe_mix3.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_uint, ctypes.c_uint,
                                   ctypes.c_uint, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_float)]
    thr = [min(int(math.floor(math.ldexp(math.exp(-4.0 * k / T), 32))), 2**32 - 1) for k in (1, 2, 3)]
    out = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    ms = ctypes.c_float()
    if L.ising_probe_mix3(out.data_ptr(), blocks, iters, thr[0], thr[1], thr[2], int(rng), int(bonds),
                          ctypes.byref(ms)) != 0:
        raise RuntimeError("mix3 probe failed")
    return blocks * 256 * iters * 32 / (ms.value * 1e-3)


def clock(blocks_per_cu=(1, 2, 4, 8), iters=20000):
    """Shader clock and per-CU issue rate of full-rate VALU ops.

    Every wave runs iters*8 independent v_xor_b32 between two shader-clock
    stamps and two real-time stamps.  Cycles per instruction per wave at a
    given occupancy give the issue rate: lane-ops per CU per cycle =
    64 * (waves per CU) / (cycles per instruction).  The shader clock is
    cycles over real time, with the real-time rate both as reported by the
    runtime and as calibrated against the launch's event time.
    """
    import numpy as np
    import torch
    L = _lib()
    L.ising_probe_clock.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_int)]
    res = {}
    for bpc in blocks_per_cu:
        blocks = CUS * bpc
        stamps = torch.zeros(blocks * 4 * 4, dtype=torch.int64, device="cuda")
        out = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
        ms, khz = ctypes.c_float(), ctypes.c_int()
        if L.ising_probe_clock(stamps.data_ptr(), out.data_ptr(), blocks, iters, ctypes.byref(ms),
                               ctypes.byref(khz)) != 0:
            raise RuntimeError("clock probe failed")
        st = stamps.view(-1, 4).cpu().numpy().astype(np.float64)
        cyc, wall, w0 = st[:, 0], st[:, 1], st[:, 3]
        span_ticks = (w0 + wall).max() - w0.min()
        calibrated_hz = span_ticks / (ms.value * 1e-3)  # real-time ticks per second (upper bound on span)
        cpi = np.median(cyc) / (iters * 8)
        waves_per_cu = 4 * bpc
        xor_rate = blocks * 256 * iters * 8 / (ms.value * 1e-3)
        res[f"{waves_per_cu}_waves_per_cu"] = {
            "event_ms": ms.value, "wall_clock_khz_reported": khz.value,
            "wall_ticks_per_s_calibrated": float(calibrated_hz),
            "shader_clock_hz_reported_rate": float(np.median(cyc / (wall / (khz.value * 1e3)))),
            "shader_clock_hz_calibrated_rate": float(np.median(cyc / (wall / calibrated_hz))),
            "cycles_per_instr_per_wave": float(cpi),
            "lane_ops_per_cu_per_cycle": 64.0 * waves_per_cu / cpi,
            "xor_lane_ops_per_s": xor_rate}
    return res


def copy_bandwidth(nbytes=1 << 30, reps=10):
    import torch
    L = _lib()
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    ms = ctypes.c_float()
    st = L.ising_probe_copy(dst.data_ptr(), src.data_ptr(), nbytes, 1, ctypes.byref(ms))
    st |= L.ising_probe_copy(dst.data_ptr(), src.data_ptr(), nbytes, reps, ctypes.byref(ms))
    if st != 0:
        raise RuntimeError("copy probe failed")
    return 2 * nbytes * reps / (ms.value * 1e-3)


if __name__ == "__main__":
    import sys
    if len(sys.argv) > 1 and sys.argv[1] == "copy":
        # calibration run for hardware traffic counters: each k_copy dispatch
        # reads and writes exactly 256 MiB
        bw = copy_bandwidth(nbytes=256 << 20, reps=3)
        print(json.dumps({"copy_dispatch_bytes_each_way": 256 << 20, "copy_bytes_per_s": bw}))
    else:
        r = measure()
        r["sweep_mix_flips_per_s"] = {str(w): mix_rate(w) for w in (32, 64)}
        r["sweep_mix_bitsliced_flips_per_s"] = {str(w): mix_rate(w, rng=1) for w in (32, 64)}
        r["sweep_mix_ordered_bonds_flips_per_s"] = {str(w): mix_rate(w, bonds=1) for w in (32, 64)}
        r["sweep_mix_bitsliced_ordered_bonds_flips_per_s"] = {str(w): mix_rate(w, rng=1, bonds=1)
                                                              for w in (32, 64)}
        r["mix3_flips_per_s"] = {"site": mix3_rate(), "bitsliced": mix3_rate(rng=1),
                                 "site_ordered_bonds": mix3_rate(bonds=1),
                                 "bitsliced_ordered_bonds": mix3_rate(rng=1, bonds=1)}
        r["clock"] = clock()
        r["copy_bytes_per_s"] = copy_bandwidth()
        print(json.dumps(r, indent=1))


def mfma_layout():
    """Check the lane layout of v_mfma_f32_16x16x32_bf16 against a host product.

    Hypothesis used by the network kernels: A (16x32) lane l holds row l%16,
    k = 8*(l//16)+i; B (32x16) lane l holds column l%16, k = 8*(l//16)+i;
    C (16x16) lane l holds column l%16, rows 4*(l//16)+i.  Returns True if it holds.
    """
    import numpy as np
    import torch
    L = _lib()
    L.ising_probe_mfma_layout.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    rng = np.random.default_rng(0)
    A = rng.integers(-8, 9, size=(16, 32)).astype(np.float32)   # exact in bf16
    B = rng.integers(-8, 9, size=(32, 16)).astype(np.float32)
    a = np.zeros((64, 8), np.float32)
    b = np.zeros((64, 8), np.float32)
    for l in range(64):
        for i in range(8):
            a[l, i] = A[l % 16, 8 * (l // 16) + i]
            b[l, i] = B[8 * (l // 16) + i, l % 16]
    to_bits = lambda m: (m.view(np.uint32) >> 16).astype(np.uint16)
    da = torch.tensor(to_bits(a).astype(np.int16).ravel(), device="cuda")
    db = torch.tensor(to_bits(b).astype(np.int16).ravel(), device="cuda")
    out = torch.zeros(64 * 4, dtype=torch.float32, device="cuda")
    if L.ising_probe_mfma_layout(da.data_ptr(), db.data_ptr(), out.data_ptr()) != 0:
        raise RuntimeError("mfma probe failed")
    o = out.cpu().numpy().reshape(64, 4)
    Cm = A @ B
    got = np.zeros((16, 16), np.float32)
    for l in range(64):
        for i in range(4):
            got[4 * (l // 16) + i, l % 16] = o[l, i]
    return bool(np.array_equal(got, Cm))


def mfma_layout_f32():
    """Check the lane layout of v_mfma_f32_16x16x4_f32 (the network's layer 1):
    A (16x4) lane l holds A[l%16][l//16]; B (4x16) lane l holds B[l//16][l%16];
    C as for the BF16 product.  Returns True if it holds."""
    import numpy as np
    import torch
    L = _lib()
    L.ising_probe_mfma_layout_f32.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    rng = np.random.default_rng(1)
    A = rng.integers(-8, 9, size=(16, 4)).astype(np.float32)
    B = rng.integers(-8, 9, size=(4, 16)).astype(np.float32)
    a = np.array([A[l % 16, l // 16] for l in range(64)], np.float32)
    b = np.array([B[l // 16, l % 16] for l in range(64)], np.float32)
    da, db = torch.tensor(a, device="cuda"), torch.tensor(b, device="cuda")
    out = torch.zeros(64 * 4, dtype=torch.float32, device="cuda")
    if L.ising_probe_mfma_layout_f32(da.data_ptr(), db.data_ptr(), out.data_ptr()) != 0:
        raise RuntimeError("mfma probe failed")
    o = out.cpu().numpy().reshape(64, 4)
    got = np.zeros((16, 16), np.float32)
    for l in range(64):
        for i in range(4):
            got[4 * (l // 16) + i, l % 16] = o[l, i]
    return bool(np.array_equal(got, A @ B))
