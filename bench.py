"""Throughput of the fused RNEA + CRBA + Jacobian chain on one MI355X.

One step = one call of the fused chain (bard_chain: inverse dynamics, mass
matrix and 4 end-effector Jacobians) over a batch of fresh synthetic
configurations of the 36-velocity-DOF humanoid tree (free root, 3-DOF waist,
1-DOF neck, two 7-DOF arms, two 6-DOF legs; FP32, batch 4096).  Input/output
sets rotate so every step reads new inputs and the working set exceeds the
256 MB Infinity Cache.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--batch B] [--no-cpu] [--no-extra]
"""

from __future__ import annotations

import argparse
import gc
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "evals/sec RNEA+CRBA+Jacobian, 23-DOF tree, batch 4096 FP32 (err vs FP64 oracle)"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_chain_humanoid_large_b4096.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2605_31481_amd", "csrc", "kernels.hip")
SPEC_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_chain_spec_humanoid_large_b4096.json")
SPEC_SRCS = [os.path.join(ROOT, "paper_2605_31481_amd", "csrc", f) for f in ("spatial.h", "specialize.cpp")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def chain_bytes_per_eval(tree, n_ee, scalar=4):
    """Algorithmic bytes of one evaluation: q, qd, qdd read; tau, M, J written."""
    return scalar * (tree.nq + 2 * tree.nv + tree.nv + tree.nv * tree.nv + n_ee * 6 * tree.nv)


def make_sets(torch, tree, B, nsets, seed):
    import synth
    sets = []
    for s in range(nsets):
        q, qd, qdd = synth.random_state(tree, B, seed + s)
        dev = [torch.from_numpy(x.T.copy()).float().cuda() for x in (q, qd, qdd)]
        n_ee = len(tree.ee_bodies)
        outs = [torch.empty((k, B), dtype=torch.float32, device="cuda")
                for k in (tree.nv, tree.nv * tree.nv, n_ee * 6 * tree.nv)]
        sets.append((dev, outs, (q, qd, qdd)))
    return sets


def time_calls(torch, calls, steps, warmup):
    """Warm up, then time exactly `steps` back-to-back calls.  One pair of HIP
    events on the launch stream brackets the timed region (events between
    launches would add work to every step); the host clock, bracketed by
    device synchronisation, gives the step rate."""
    n = len(calls)
    for k in range(warmup):
        calls[k % n]()
    st = torch.cuda.Event(enable_timing=True)
    en = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    # Python's collector is paused while timing: its pauses (hundreds of
    # microseconds) would otherwise land between launches at random
    gc.collect()
    gc.disable()
    try:
        t0 = time.perf_counter()
        st.record()
        for k in range(steps):
            calls[k % n]()
        en.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    finally:
        gc.enable()
    return wall, st.elapsed_time(en) / steps


def time_graph(torch, make_calls, replays):
    """Capture one pass over the rotation sets in a HIP graph and replay it.
    `make_calls` binds the calls to the stream current when it runs, so the
    launches made during capture land on the capturing stream."""
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for c in make_calls():
            c()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        calls = make_calls()
        for c in calls:
            c()
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(replays):
        g.replay()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / (replays * len(calls))


def parity_sample(tree, sets, n_sample=256):
    """Per-entry error of the last timed outputs of set 0 against the FP64
    oracle on sampled instances, under the tests' contract: tau and M entries
    against atol + rtol max(|ref|, S) with S the transmitted-wrench scale
    (tau) or sqrt(M_ii M_jj) (M), Jacobian entries against their column's
    largest entry.  Also reports the normwise-per-block ratio."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from oracle import OracleModel
    from parity_util import TOL, column_scale, entry_scales
    import synth
    (dev, outs, host) = sets[0]
    q, qd, qdd = (synth.to_fp32_grid(x) for x in host)
    B = q.shape[0]
    idx = np.random.default_rng(0).choice(B, min(n_sample, B), replace=False)
    q, qd, qdd = q[idx], qd[idx], qdd[idx]
    om = OracleModel.from_tree(tree)
    rt, rM, rJ = om.chain(q, qd, qdd, tree.ee_bodies)
    st, sm = entry_scales(om, tree, q, qd, qdd)
    rtol, atol = TOL["float32"]
    n = len(idx)
    g = [o.cpu().double().numpy().T[idx] for o in outs]
    refs = (rt, rM.reshape(n, -1), rJ.reshape(n, -1))
    scales = (st, sm, column_scale(rJ).reshape(n, -1))
    per_entry = {}
    for lbl, gg, r, sc in zip(("tau", "M", "J"), g, refs, scales):
        per_entry[lbl] = float((np.abs(gg - r) / (atol + rtol * np.maximum(np.abs(r), sc))).max())
    normwise = max(float((np.abs(gg - r).max(1) / (atol + rtol * np.abs(r).max(1))).max()) for gg, r in zip(g, refs))
    worst = max(per_entry.values())
    return {"max_err_over_tol": worst, "per_entry": per_entry, "normwise_per_block": normwise,
            "instances": int(n),
            "tolerance": "per entry |gpu-ref| <= 1e-6 + 1e-5 max(|ref|, S): S = transmitted-wrench scale (tau), "
                         "sqrt(M_ii M_jj) (M), column max (J)",
            "pass": worst <= 1.0}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(tree, target_s=10.0, max_s=30.0):
    """The FP64 oracle (untuned) on a bounded sample of the same workload."""
    from oracle import OracleModel
    import synth
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    om = OracleModel.from_tree(tree)
    chunk = 4096
    q, qd, qdd = synth.random_state(tree, chunk, 7777)
    om.chain(q[:64], qd[:64], qdd[:64], tree.ee_bodies, threads=threads)
    done, t0 = 0, time.perf_counter()
    while True:
        om.chain(q, qd, qdd, tree.ee_bodies, threads=threads)
        done += chunk
        el = time.perf_counter() - t0
        if el >= target_s or el >= max_s:
            break
    # one thread, as a sequential loop over configurations
    one, t1 = 0, time.perf_counter()
    while True:
        om.chain(q[:512], qd[:512], qdd[:512], tree.ee_bodies, threads=1)
        one += 512
        el1 = time.perf_counter() - t1
        if el1 >= target_s / 2:
            break
    return {"value": done / el, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} configurations of the same tree (RNEA+CRBA+4-EE Jacobian, FP64), "
                      f"{el:.1f} s on {threads} OpenMP threads",
            "value_1_thread": one / el1, "cpu_model": cpu_model()}


def _rate(torch, calls, steps, warmup=10):
    wall, kavg = time_calls(torch, calls, steps, warmup)
    return wall / steps, kavg * 1e-3


def bench_sweep(torch, bard, m, tree, bpe):
    """The fused chain on the 36-DOF humanoid over batch sizes 64 .. 262,144:
    evaluations per second from one event pair around back-to-back launches,
    rotating input/output sets up to 512 MB (at most 64 sets, so the smallest
    batches stay cache-resident and launch-bound)."""
    ee = tree.ee_bodies
    out = {}
    for B in (64, 256, 1024, 4096, 16384, 65536, 262144):
        nsets = max(1, min(64, math.ceil(512e6 / (bpe * B))))
        sets = make_sets(torch, tree, B, nsets, 9000 + B)
        calls = [m.bind_chain(d[0], d[1], d[2], ee, tuple(o)) for (d, o, _) in sets]
        n = max(30, min(300, 4_000_000 // B))
        wall, kavg = time_calls(torch, calls, n, 10)
        out[f"sweep_B{B}_evals_per_s"] = B / (kavg * 1e-3)
        out[f"sweep_B{B}_kernel_us"] = kavg * 1e3
        out[f"sweep_B{B}_hbm_frac"] = bpe * B / (kavg * 1e-3) / 1e9 / HBM_PEAK_GBS
        del sets, calls
        torch.cuda.empty_cache()
    return out


# FP32 vector peak of the spec sheet, 157.3 TFLOP/s (256 CU x 2.4 GHz x 256 FLOP per
# CU per clock).  Plain (unpacked) FMAs reach it: the peak probe measures
# 122-131 TFLOP/s with packed FP32 instructions off, as the library builds.
VALU_PEAK_FP32 = 157.3e12


def op_work(tree, n_ee, op):
    """(algorithmic bytes, FLOP) of one evaluation of one operator in FP32.
    Bytes: the inputs read and the outputs written.  FLOP: the per-body FMA
    model (2 FLOP per FMA) -- joint transform 24, pose composition 36, RNEA
    forward 130 and backward 33, ABA 380 -- for the operators bound by
    arithmetic; None for the memory-bound ones."""
    n, nq, nv = tree.n_bodies, tree.nq, tree.nv
    if op == "fk":
        return 4 * (nq + 12 * n), 2 * n * (24 + 36)
    if op == "jacobian":
        return 4 * (nq + 6 * nv * n_ee), None
    if op == "rnea":
        return 4 * (nq + 3 * nv), 2 * n * (24 + 130 + 33)
    if op == "crba":
        return 4 * (nq + nv * nv), None
    if op == "path":  # one end effector's pose and Jacobian from its path's coordinates
        import synth
        e = tree.ee_bodies[0]
        nqp = 0
        while e >= 0:
            nqp += 7 if tree.joint_type[e] == synth.FREE else 1
            e = tree.parent[e]
        return 4 * (nqp + 12 + 6 * nv), None
    if op == "aba":
        return 4 * (nq + 3 * nv), 2 * n * (24 + 380)
    raise ValueError(op)


def bench_operators(torch, bard):
    """Each plain operator alone (FK, the 4-end-effector Jacobian, RNEA and
    CRBA with the generic and the model-specialised kernels; ABA; and the standalone pose and Jacobian
    of the first end effector's path) on the 36-DOF humanoid at B = 4096 and 16384 and on the 7-DOF chain
    at B = 4096, FP32, rotating input/output sets past 512 MB.  Per operator:
    evaluations per second from the kernel time, the HBM fraction of its
    algorithmic bytes, and for RNEA and ABA the FP32 VALU fraction of the
    per-body FLOP model.  Then the 23-DOF humanoid at B = 16384: fused chain,
    three plain launches and graph replay."""
    import synth
    out = {}
    for name, B in (("humanoid_large", 4096), ("humanoid_large", 16384), ("chain7", 4096)):
        tree = synth.tree_by_name(name)
        m = bard.Model.from_tree(tree)
        ee = tree.ee_bodies
        mr = bard.Model.from_tree(tree)   # its rnea(), crba(), jacobian() calls routed to specialised kernels
        mr.specialize_rnea()
        mr.specialize_op("crba")
        mr.specialize_op("jacobian", ee=ee)
        mr.specialize_op("fk")
        per_eval = 4 * (tree.nq + 4 * tree.nv + 12 * tree.n_bodies + tree.nv * tree.nv + 6 * tree.nv * len(ee))
        nsets = max(3, min(64, math.ceil(512e6 / (per_eval * B))))
        sets = []
        for k in range(nsets):
            q, qd, qdd = synth.random_state(tree, B, 11000 + k)
            d = [torch.from_numpy(x.T.copy()).float().cuda() for x in (q, qd, qdd)]
            o = {"fk": torch.empty((12 * tree.n_bodies, B), device="cuda"),
                 "jacobian": torch.empty((6 * tree.nv * len(ee), B), device="cuda"),
                 "rnea": torch.empty((tree.nv, B), device="cuda"),
                 "crba": torch.empty((tree.nv * tree.nv, B), device="cuda"),
                 "aba": torch.empty((tree.nv, B), device="cuda"),
                 "path_pose": torch.empty((12, B), device="cuda"),
                 "path_J": torch.empty((6 * tree.nv, B), device="cuda")}
            sets.append((d, o))
        binders = {"fk": lambda d, o: m.bind_fk(d[0], o["fk"]),
                   "fk_specialized": lambda d, o: mr.bind_fk(d[0], o["fk"]),
                   "jacobian": lambda d, o: m.bind_jacobian(d[0], ee, o["jacobian"]),
                   "jacobian_specialized": lambda d, o: mr.bind_jacobian(d[0], ee, o["jacobian"]),
                   "rnea": lambda d, o: m.bind_rnea(d[0], d[1], d[2], o["rnea"]),
                   "rnea_specialized": lambda d, o: mr.bind_rnea(d[0], d[1], d[2], o["rnea"]),
                   "crba": lambda d, o: m.bind_crba(d[0], o["crba"]),
                   "crba_specialized": lambda d, o: mr.bind_crba(d[0], o["crba"]),
                   "aba": lambda d, o: m.bind_aba(d[0], d[1], d[2], o["aba"]),   # qdd's values as torques
                   "path": lambda d, o: m.bind_path_kinematics(d[0], ee[0], o["path_pose"], o["path_J"],
                                                               frame=bard.LOCAL_WORLD_ALIGNED)}
        n = max(100, min(1000, 4_000_000 // B))
        for op, bind in binders.items():
            calls = [bind(d, o) for (d, o) in sets]
            _, kavg = time_calls(torch, calls, n, 10)
            t = kavg * 1e-3
            nbytes, flops = op_work(tree, len(ee), op.replace("_specialized", ""))
            key = f"op_{name}_B{B}_{op}"
            out[key + "_evals_per_s"] = B / t
            out[key + "_kernel_us"] = kavg * 1e3
            out[key + "_hbm_frac"] = nbytes * B / t / 1e9 / HBM_PEAK_GBS
            if flops is not None:
                out[key + "_valu_frac"] = flops * B / t / VALU_PEAK_FP32
        del sets
        torch.cuda.empty_cache()
    # the standalone path kinematics where it is bound by HBM: the humanoid's
    # first end effector at B = 262144, both frames
    tree = synth.humanoid_large()
    m = bard.Model.from_tree(tree)
    B = 262144
    nbytes, _ = op_work(tree, 1, "path")
    sets = []
    for k in range(3):
        q = synth.random_state(tree, B, 11500 + k)[0]
        sets.append((torch.from_numpy(q.T.copy()).float().cuda(), torch.empty((12, B), device="cuda"),
                     torch.empty((6 * tree.nv, B), device="cuda")))
    for frame, fname in ((bard.WORLD, "world"), (bard.LOCAL_WORLD_ALIGNED, "lwa")):
        calls = [m.bind_path_kinematics(q, tree.ee_bodies[0], po, J, frame=frame) for (q, po, J) in sets]
        _, kavg = time_calls(torch, calls, 200, 10)
        key = f"op_humanoid_large_B{B}_path_{fname}"
        out[key + "_kernel_us"] = kavg * 1e3
        out[key + "_evals_per_s"] = B / (kavg * 1e-3)
        out[key + "_hbm_frac"] = nbytes * B / (kavg * 1e-3) / 1e9 / HBM_PEAK_GBS
    del sets
    torch.cuda.empty_cache()
    # the 23-velocity-DOF humanoid at B = 16384: fused, plain and graph forms
    ts = synth.humanoid_small()
    ms = bard.Model.from_tree(ts)
    B = 16384
    bpe = chain_bytes_per_eval(ts, len(ts.ee_bodies))
    sets = make_sets(torch, ts, B, max(4, math.ceil(512e6 / (bpe * B))), 12000)
    mk = lambda: [ms.bind_chain(d[0], d[1], d[2], ts.ee_bodies, tuple(o)) for (d, o, _) in sets]
    calls = mk()
    _, kf = time_calls(torch, calls, 200, 10)
    plain = [(ms.bind_rnea(d[0], d[1], d[2], o[0]), ms.bind_crba(d[0], o[1]), ms.bind_jacobian(d[0], ts.ee_bodies, o[2]))
             for (d, o, _) in sets]
    _, kp = time_calls(torch, [(lambda t=t: (t[0](), t[1](), t[2]())) for t in plain], 200, 10)
    out["nv23_B16384_chain_evals_per_s"] = B / (kf * 1e-3)
    out["nv23_B16384_chain_hbm_frac"] = bpe * B / (kf * 1e-3) / 1e9 / HBM_PEAK_GBS
    out["nv23_B16384_plain_3_launches_evals_per_s"] = B / (kp * 1e-3)
    out["nv23_B16384_graph_replay_evals_per_s"] = B / time_graph(torch, mk, 20)
    del sets, calls, plain
    torch.cuda.empty_cache()
    return out


def measure_peaks(torch):
    """The peaks the roofline fractions are taken against, measured on this
    GPU: FP32 VALU FMA throughput from the peak probe (eight independent FMA
    chains per lane, packed FP32 off as in the library) and HBM bandwidth of a
    1 GiB device-to-device copy (bytes read + written)."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2605_31481_amd", "libbard_peaks.so"))
    lib.bard_peak_fma_fp32.restype = ctypes.c_double
    lib.bard_peak_fma_fp32.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    blocks, iters = 256 * 32, 256
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    flops = lib.bard_peak_fma_fp32(ctypes.c_void_p(out.data_ptr()), blocks, iters, stream)
    if flops < 0:
        raise RuntimeError("peak probe launch failed")
    best = 0.0
    for _ in range(5):
        st, en = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        st.record()
        lib.bard_peak_fma_fp32(ctypes.c_void_p(out.data_ptr()), blocks, iters, stream)
        en.record()
        torch.cuda.synchronize()
        best = max(best, flops / (st.elapsed_time(en) * 1e-3))
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    bw = 0.0
    for _ in range(5):
        st, en = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        st.record()
        dst.copy_(src)
        en.record()
        torch.cuda.synchronize()
        bw = max(bw, 2 * src.numel() * 4 / (st.elapsed_time(en) * 1e-3))
    del src, dst, out
    torch.cuda.empty_cache()
    return {"peak_fp32_fma_tflops_measured": best / 1e12, "peak_fp32_vector_tflops_spec": VALU_PEAK_FP32 / 1e12,
            "peak_hbm_copy_gbs_measured": bw / 1e9, "peak_hbm_gbs_spec": HBM_PEAK_GBS}


def bench_specialized(torch, bard):
    """Model-specialised chain kernels (hipRTC, constants as literals) against
    the generic kernel: the four forms (split over waves by limbs, dual:
    split with torques and mass matrix + Jacobians in two workgroups, triple:
    torques, mass matrix and Jacobians in three, and the whole tree per
    wave) on the 36-DOF and 23-DOF humanoids and the 7-DOF chain at
    B = 1024 .. 262,144, rotating sets past 512 MB; then the tiers
    bard_chain_autotune routes to each form; then the specialised
    forward-dynamics (ABA) kernel against the generic one at the same
    batches, and the tiers bard_aba_autotune routes to it."""
    import synth
    out = {}
    for name, batches in (("humanoid_large", (1024, 4096, 16384, 65536, 262144)),
                          ("humanoid_small", (1024, 4096, 16384, 65536)), ("chain7", (1024, 4096, 16384, 65536))):
        tree = synth.tree_by_name(name)
        m = bard.Model.from_tree(tree)
        ee = tree.ee_bodies
        bpe = chain_bytes_per_eval(tree, len(ee))
        forms = bard.SPEC_FORMS
        for f in forms:
            m.specialize(ee, route=False, form=f)
            info = m.specialized_info(ee, form=f)
            for k in ("compile_s", "vgprs", "scratch_bytes", "waves"):
                out[f"spec_{name}_{f}_{k}"] = info[k]
        for B in batches:
            nsets = max(2, min(64, math.ceil(512e6 / (bpe * B))))
            sets = make_sets(torch, tree, B, nsets, 13000 + B)
            calls = [m.bind_chain(d[0], d[1], d[2], ee, tuple(o)) for (d, o, _) in sets]
            n = max(30, min(400, 2_000_000 // B))
            key = f"spec_{name}_B{B}"
            for f in forms:
                m.specialize(ee, route=False, form=f)
            _, kg = time_calls(torch, calls, n, 5)
            out[key + "_generic_us"] = kg * 1e3
            for f in forms:
                m.specialize(ee, route=True, form=f)
                _, ks = time_calls(torch, calls, n, 5)
                out[key + f"_{f}_us"] = ks * 1e3
                out[key + f"_{f}_hbm_frac"] = bpe * B / (ks * 1e-3) / 1e9 / HBM_PEAK_GBS
            del sets, calls
            torch.cuda.empty_cache()
        out[f"spec_{name}_autotuned_first_batch"] = m.autotune_chain(ee)
        out[f"spec_{name}_autotuned_tiers"] = {f: m.specialized_info(ee, form=f)["route_tiers"] for f in forms}
        # forward dynamics (ABA): generic and specialised kernel on rotating sets
        m.specialize_aba(route=False)
        info = m.specialized_aba_info()
        out[f"spec_aba_{name}_vgprs"] = info["vgprs"]
        out[f"spec_aba_{name}_scratch_bytes"] = info["scratch_bytes"]
        out[f"spec_aba_{name}_compile_s"] = info["compile_s"]
        abpe = 4 * (tree.nq + 3 * tree.nv)
        for B in batches:
            nsets = max(2, min(64, math.ceil(512e6 / (abpe * B))))
            sets = []
            for k in range(nsets):
                q, qd, _ = synth.random_state(tree, B, 14000 + B + k)
                d = [torch.from_numpy(x.T.copy()).float().cuda() for x in (q, qd, qd)]   # qd's values as torques
                sets.append((d, torch.empty((tree.nv, B), device="cuda")))
            calls = [m.bind_aba(d[0], d[1], d[2], o) for (d, o) in sets]
            n = max(30, min(400, 2_000_000 // B))
            key = f"spec_aba_{name}_B{B}"
            m.specialize_aba(route=False)
            _, kg = time_calls(torch, calls, n, 5)
            m.specialize_aba(route=True)
            _, ks = time_calls(torch, calls, n, 5)
            out[key + "_generic_us"] = kg * 1e3
            out[key + "_specialized_us"] = ks * 1e3
            out[key + "_specialized_evals_per_s"] = B / (ks * 1e-3)
            del sets, calls
            torch.cuda.empty_cache()
        out[f"spec_aba_{name}_autotuned_first_batch"] = m.autotune_aba()
        out[f"spec_aba_{name}_autotuned_tiers"] = m.specialized_aba_info()["route_tiers"]
    return out


def bench_plan(torch, bard, steps):
    """Five random trees (7, 11, 12, 18, 23 DOF; batches 512..8192 = 15,872
    instances; RNEA + CRBA + tip Jacobians): one plan with the configuration
    the autotuner picks (generic work-item kernel or the generated
    multi-tree kernel), device time from graph replay, against the untuned
    default and five separate chain launches (graph replay too).  Every run
    reads and writes the same arrays (58 MB, within the 256 MB Infinity
    Cache), as a captured plan run must use the io of the run before it."""
    import synth
    trees = synth.multi_trees()
    batches = synth.MULTI_BATCHES
    models = [bard.Model.from_tree(t) for t in trees]
    plan = bard.Plan(models, batches)
    ins = []
    for k, (t, B) in enumerate(zip(trees, batches)):
        q, qd, qdd = synth.random_state(t, B, 6000 + k)
        ins.append(tuple(torch.from_numpy(x.T.copy()).float().cuda() for x in (q, qd, qdd)))
    default_cfg = plan.config
    plan.run(ins)
    torch.cuda.synchronize()
    t_def, k_def = _rate(torch, [lambda: plan.run(ins)], 50)
    plan.autotune()
    total = sum(batches)
    nbytes = sum(4 * B * (t.nq + 3 * t.nv + t.nv * t.nv + 6 * t.nv * len(plan.ee(k)))
                 for k, (t, B) in enumerate(zip(trees, batches)))
    plan.run(ins)
    plan.run(ins)
    torch.cuda.synchronize()
    n = max(50, steps // 4)
    # device time per run from replays of a graph of 20 runs (an eager run
    # costs tens of microseconds of Python and ctypes, more than the kernel);
    # the eager rate beside it includes that host time
    g_plan = time_graph(torch, lambda: [lambda: plan.run(ins)] * 20, 20)
    t_plan, _ = _rate(torch, [lambda: plan.run(ins)], n)
    outs = [tuple(torch.empty((K, B), device="cuda") for K in (t.nv, t.nv * t.nv, 6 * t.nv * len(plan.ee(k))))
            for k, (t, B) in enumerate(zip(trees, batches))]
    mk_sep = lambda: [m.bind_chain(i[0], i[1], i[2], plan.ee(k), o)
                      for k, (m, i, o) in enumerate(zip(models, ins, outs))]
    g_sep = time_graph(torch, lambda: mk_sep() * 4, 20) * 5
    out = {"plan5_evals_per_s": total / g_plan, "plan5_gpu_us": g_plan * 1e6,
           "plan5_hbm_frac": nbytes / g_plan / 1e9 / HBM_PEAK_GBS, "plan5_config": plan.config,
           "plan5_eager_evals_per_s": total / t_plan,
           "plan5_default_config": default_cfg, "plan5_default_eager_us": k_def * 1e6,
           "separate5_evals_per_s": total / g_sep, "separate5_gpu_us": g_sep * 1e6}
    if plan.config["fusion"] == 3:
        out["plan5_generated_kernel"] = plan.specialized_info()
    return out


def bench_adjoints(torch, bard, steps):
    """RNEA adjoint on the identification workload (11-DOF quadruped, 4096
    trajectories x 200 steps = 819,200 instances, FP32) with the batch-summed
    inertial-parameter gradient; FK adjoint at the same size."""
    import synth
    tree = synth.quadruped_spine()
    m = bard.Model.from_tree(tree)
    q, qd, qdd = synth.sinusoid_trajectories(tree, 4096, 200, seed=4242)
    B = q.shape[0]
    dev = [torch.from_numpy(x.T.copy()).float().cuda() for x in (q, qd, qdd)]
    tb = torch.randn((tree.nv, B), device="cuda")
    n = max(20, steps // 20)
    t_v, k_v = _rate(torch, [lambda: m.rnea_vjp(dev[0], dev[1], dev[2], tb)], n, 3)
    bytes_v = 4 * B * (tree.nq + 3 * tree.nv + tree.nq + 2 * tree.nv)
    pb = torch.randn((12 * tree.n_bodies, B), device="cuda")
    t_f, k_f = _rate(torch, [lambda: m.fk_vjp(dev[0], pb)], n, 3)
    bytes_f = 4 * B * (tree.nq + 12 * tree.n_bodies + tree.nq)
    return {"rnea_vjp_819200_evals_per_s": B / t_v, "rnea_vjp_819200_gpu_us": k_v * 1e6,
            "rnea_vjp_819200_hbm_frac": bytes_v / k_v / 1e9 / HBM_PEAK_GBS,
            "fk_vjp_819200_evals_per_s": B / t_f, "fk_vjp_819200_gpu_us": k_f * 1e6,
            "fk_vjp_819200_hbm_frac": bytes_f / k_f / 1e9 / HBM_PEAK_GBS}


def sysid_data():
    import synth
    tree = synth.quadruped_spine()
    return tree, [synth.to_fp32_grid(x) for x in synth.random_state(tree, 10000, 9100)]


def sysid_reference():
    """The oracle's part of the identification experiment (run in the oracle
    leg): the torques at the true parameters, and the regressor of the masses
    -- with pi(m) = A + m D per link, tau = RNEA(A) + sum_k m_k RNEA(D_k) --
    from which each seed's least-squares optimum, the best any optimiser can
    reach on that noisy data, is solved directly."""
    from oracle import OracleModel
    from paper_2605_31481_amd.sysid import mass_map
    tree, (q, qd, qdd) = sysid_data()
    om = OracleModel.from_tree(tree)
    A, D, m_true = mass_map(tree.inertia)
    tau_a = om.rnea(q, qd, qdd, inertia=A)
    cols = []
    for k in range(tree.n_bodies):
        pi = np.zeros_like(A)
        pi[k] = D[k]
        cols.append(om.rnea(q, qd, qdd, inertia=pi).ravel())
    return {"tau": om.rnea(q, qd, qdd), "tau_a": tau_a, "phi": np.stack(cols, axis=1), "m_true": m_true}


def bench_sysid(torch, bard, ref):
    """Mass identification (Sec. 4.3's experiment) on 10,000 random
    configurations of the 11-DOF quadruped: torques from the true parameters
    by the FP64 oracle plus 5% Gaussian noise per joint, masses started 30%
    away from the truth, L-BFGS, 10 seeds; in FP32 with and without the
    diagonal scaling of the masses, and in FP64.  The least-squares optimum of
    each seed's data gives the noise floor of the error and the optimiser's
    remaining distance."""
    from paper_2605_31481_amd import sysid
    tree, host = sysid_data()
    m = bard.Model.from_tree(tree)
    out = {}
    phi, tau_a, m_true = ref["phi"], ref["tau_a"], ref["m_true"]
    for label, dtype, pre in (("fp32", torch.float32, True), ("fp32_unscaled", torch.float32, False),
                              ("fp64", torch.float64, True)):
        q, qd, qdd = (torch.from_numpy(x.T.copy()).to(dtype).cuda() for x in host)
        tau_true = torch.from_numpy(ref["tau"].T.copy()).to(dtype).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = sysid.identify(m, tree.inertia, q, qd, qdd, seeds=range(10), noise=0.05, max_iter=60,
                             tau_true=tau_true, precondition=pre)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        per_seed = res["rel_error"].mean(axis=1) * 100
        dist, floor = [], []
        for k in range(10):
            meas = sysid.noisy_torques(tau_true, 0.05, 7000 + k).double().cpu().numpy().T
            m_ls = np.linalg.lstsq(phi, (meas - tau_a).ravel(), rcond=None)[0]
            dist.append(float(np.abs(res["masses"][k] - m_ls).max() / np.abs(m_ls).max()))
            floor.append(float((np.abs(m_ls - m_true) / m_true).max()))
        out[f"sysid_{label}_mean_mass_error_pct"] = float(per_seed.mean())
        out[f"sysid_{label}_std_over_seeds_pct"] = float(per_seed.std())
        out[f"sysid_{label}_worst_link_error_pct"] = float(res["rel_error"].max() * 100)
        out[f"sysid_{label}_iterations_mean"] = float(np.mean(res["iterations"]))
        out[f"sysid_{label}_evaluations_total"] = int(np.sum(res["evaluations"]))
        out[f"sysid_{label}_seconds_10_seeds"] = el
        out[f"sysid_{label}_max_distance_to_least_squares"] = max(dist)
        out[f"sysid_{label}_least_squares_worst_link_error_pct"] = 100 * max(floor)
    return out


def bench_workspace(torch, bard, steps):
    """Cache patterns of the workspace tiers, B = 4096 FP32, on the 7-DOF
    chain and the 36-DOF humanoid.  One step is FK, Jacobian, CRBA and RNEA on
    one state, as four calls.  Patterns: P0 every input new (all tiers miss),
    P1 the same q, qd, qdd again, P2 the same q with a new qd.  Policies: no
    workspace, the kinematics tier alone, and kinematics + mass + bias tiers.
    Each pattern's last outputs are compared with cold calls (no workspace) on
    the same inputs: the largest difference relative to the output's size
    (zero where the tier returns the cold call's bits)."""
    import synth
    out = {}
    for name in ("chain7", "humanoid_large"):
        tree = synth.tree_by_name(name)
        m = bard.Model.from_tree(tree)
        B = 4096
        hq, hqd, hqdd = synth.random_state(tree, B, 7000)
        _, hqd2, _ = synth.random_state(tree, B, 7001)
        q, qd, qdd, qd2 = (torch.from_numpy(synth.to_fp32_grid(x).T.copy()).float().cuda()
                           for x in (hq, hqd, hqdd, hqd2))
        ee = tree.ee_bodies
        outs = dict(fk=torch.empty((12 * tree.n_bodies, B), device="cuda"),
                    j=torch.empty((6 * len(ee) * tree.nv, B), device="cuda"),
                    M=torch.empty((tree.nv * tree.nv, B), device="cuda"), tau=torch.empty((tree.nv, B), device="cuda"))
        ctr = [10]

        def step(w, pattern):
            ctr[0] += 1
            qt = ctr[0] if pattern == "P0" else 1
            dt = 1 if pattern == "P1" else ctr[0]
            v = qd if (pattern != "P2" or ctr[0] % 2) else qd2
            m.fk(q, out=outs["fk"], ws=w, q_tag=qt)
            m.jacobian(q, ee, out=outs["j"], ws=w, q_tag=qt)
            m.crba(q, out=outs["M"], ws=w, q_tag=qt)
            m.rnea(q, v, qdd, out=outs["tau"], ws=w, q_tag=qt, qd_tag=dt)
            return v

        n = max(50, steps // 4)
        for label, pol in (("no_ws", None), ("kin", 1), ("all", 7)):
            for pattern in ("P0", "P1", "P2"):
                if pol is None and pattern != "P0":
                    continue
                w = bard.Workspace(m, B, policy=pol) if pol is not None else None
                t, k = _rate(torch, [lambda: step(w, pattern)], n)
                v = step(w, pattern)
                cold = (m.fk(q), m.jacobian(q, ee), m.crba(q), m.rnea(q, v, qdd))
                torch.cuda.synchronize()
                diff = max(float(((a - c).abs().max() / c.abs().max().clamp_min(1e-30)).item())
                           for a, c in zip((outs["fk"], outs["j"], outs["M"], outs["tau"]), cold))
                key = f"{name}_{label}_{pattern}"
                out[key + "_gpu_us"] = k * 1e6
                out[key + "_rel_diff_vs_cold"] = diff
    return out


def spec_source_sha(m, ee, form):
    """SHA-256 of what a specialised kernel is built and launched from: its
    generated source, the device header it includes and the generator."""
    h = hashlib.sha256(m.specialized_source(ee, form=form).encode())
    for f in SPEC_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def traffic_if_current(spec_sha=None):
    """The counted HBM bytes per launch of the timed kernel, if the record was
    taken on the current source (None otherwise)."""
    path = SPEC_TRAFFIC_FILE if spec_sha else TRAFFIC_FILE
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    sha = spec_sha or hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if rec.get("kernels_sha256") != sha:
        return None
    return rec.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--only", default="",
                    help="comma-separated subset of the extras to run (chainforms, peaks, ops, sweep, specialized, "
                         "plan, adjoints, workspace, sysid), e.g. for a profile of one group")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run 3 plain device-to-device copies of this many MiB (a kernel of known traffic "
                         "that calibrates the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (a batch would shard "
              "across GPUs by instance ranges with no exchange). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2605_31481_amd import bard

    torch.cuda.set_device(0)
    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: 3 copies of {args.copy_mib} MiB")
        del src, dst
    tree = synth.humanoid_large()
    m = bard.Model.from_tree(tree)
    B = args.batch
    ee = tree.ee_bodies
    bpe = chain_bytes_per_eval(tree, len(ee))
    per_call = bpe * B
    nsets = max(14, math.ceil(512e6 / per_call))
    log(f"[bench] workload humanoid_large nv={tree.nv} B={B} bytes/call={per_call/1e6:.1f} MB sets={nsets}")
    sets = make_sets(torch, tree, B, nsets, 2002)
    # bard_chain_autotune (untimed, once) routes each batch tier to the fastest
    # of the generic kernel and the two specialised forms
    t0 = time.perf_counter()
    first = m.autotune_chain(ee)
    tiers = {f: m.specialized_info(ee, form=f)["route_tiers"] for f in bard.SPEC_FORMS}
    tier = sum(B >= t for t in bard.SPEC_TIERS[1:])
    route = next((f for f, bits in tiers.items() if (bits >> tier) & 1), "generic")
    spec_sha = spec_source_sha(m, ee, route) if route != "generic" else None
    kernel = {"generic": "tree_kernel<float, RNEA|CRBA|JAC>",
              "split": f"bard_spec_chain (specialised, split over {m.specialized_info(ee)['waves']} waves)",
              "whole": "bard_spec_chain (specialised, whole tree per wave)",
              "dual": f"bard_spec_chain (specialised, split over {m.specialized_info(ee, form='dual')['waves']} waves, "
                      "torques and mass matrix + Jacobians in two workgroups)",
              "triple": f"bard_spec_chain (specialised, split over {m.specialized_info(ee, form='triple')['waves']} "
                        "waves, torques, mass matrix and Jacobians in three workgroups)"}[route]
    log(f"[bench] autotune {time.perf_counter() - t0:.1f} s: tiers {tiers}, first specialised batch {first}; "
        f"B={B} runs {kernel}")
    def make_calls():
        return [m.bind_chain(d[0], d[1], d[2], ee, tuple(o)) for (d, o, _) in sets]
    calls = make_calls()

    wall, kavg = time_calls(torch, calls, args.steps, args.warmup)
    value = B * args.steps / wall
    achieved = per_call / (kavg * 1e-3) / 1e9
    log(f"[bench] chain: {value:.4g} evals/s, kernel avg {kavg*1e3:.2f} us")

    extra = {"autotune_route_tiers": tiers, "autotune_first_specialised_batch": first}
    if route != "generic":
        # the generic kernel on the same sets, for comparison
        mg = bard.Model.from_tree(tree)
        gcalls = [mg.bind_chain(d[0], d[1], d[2], ee, tuple(o)) for (d, o, _) in sets]
        gw, gk = time_calls(torch, gcalls, args.steps, args.warmup)
        extra["generic_kernel_evals_per_s"] = B * args.steps / gw
        extra["generic_kernel_us"] = gk * 1e3
        extra["generic_kernel_hbm_frac"] = per_call / (gk * 1e-3) / 1e9 / HBM_PEAK_GBS
        log(f"[bench] generic chain kernel on the same sets: {gk*1e3:.2f} us")
        # the routed calls write the outputs the parity leg samples
        for c in calls[:nsets]:
            c()
        torch.cuda.synchronize()
    only = set(x for x in args.only.split(",") if x)
    want = lambda k: not args.no_extra and (not only or k in only)
    if want("chainforms"):
        # plain per-operator kernels (three launches) on the same sets
        plain = []
        for (d, o, _) in sets:
            plain.append((m.bind_rnea(d[0], d[1], d[2], o[0]), m.bind_crba(d[0], o[1]),
                          m.bind_jacobian(d[0], ee, o[2])))
        pcalls = [(lambda t=t: (t[0](), t[1](), t[2]())) for t in plain]
        pw, pk = time_calls(torch, pcalls, max(100, args.steps // 4), 10)
        extra["plain_3_launches_evals_per_s"] = B * max(100, args.steps // 4) / pw
        extra["graph_replay_evals_per_s"] = B / time_graph(torch, make_calls, max(5, args.steps // nsets))
        # same buffers every call (working set in the Infinity Cache)
        sw, sk = time_calls(torch, calls[:1], max(100, args.steps // 4), 10)
        extra["same_buffers_kernel_us"] = sk * 1e3
        # the paper's protocol: median of 100 individually timed calls (an
        # event pair around each call, the device drained between calls), and
        # the host time of one call through the C ABI (the launch is
        # asynchronous, so this is the marshalling and launch cost)
        per_call, host = [], []
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(100)]
        for k in range(100):
            torch.cuda.synchronize()
            ev[k][0].record()
            h0 = time.perf_counter()
            calls[k % nsets]()
            host.append(time.perf_counter() - h0)
            ev[k][1].record()
        torch.cuda.synchronize()
        per_call = [a.elapsed_time(b) * 1e3 for a, b in ev]
        extra["median_of_100_calls_us"] = float(np.median(per_call))
        extra["host_us_per_call"] = float(np.median(host)) * 1e6
        # larger batch
        B2 = 16384
        sets2 = make_sets(torch, tree, B2, max(4, math.ceil(512e6 / (bpe * B2))), 4002)
        calls2 = [m.bind_chain(d[0], d[1], d[2], ee, tuple(o)) for (d, o, _) in sets2]
        w2, k2 = time_calls(torch, calls2, max(100, args.steps // 4), 10)
        extra["batch16384_evals_per_s"] = B2 * max(100, args.steps // 4) / w2
        extra["batch16384_kernel_us"] = k2 * 1e3
        extra["batch16384_hbm_frac"] = bpe * B2 / (k2 * 1e-3) / 1e9 / HBM_PEAK_GBS
        del sets2, calls2
        # the 23-velocity-DOF companion tree, autotuned as the headline is
        ts = synth.humanoid_small()
        ms = bard.Model.from_tree(ts)
        extra["nv23_autotuned_first_specialised_batch"] = ms.autotune_chain(ts.ee_bodies)
        bpe_s = chain_bytes_per_eval(ts, len(ts.ee_bodies))
        sets3 = make_sets(torch, ts, B, max(14, math.ceil(512e6 / (bpe_s * B))), 5002)
        calls3 = [ms.bind_chain(d[0], d[1], d[2], ts.ee_bodies, tuple(o)) for (d, o, _) in sets3]
        w3, k3 = time_calls(torch, calls3, args.steps, 10)
        extra["nv23_tree_evals_per_s"] = B * args.steps / w3
        extra["nv23_tree_kernel_us"] = k3 * 1e3
        del sets3, calls3
    if want("peaks"):
        extra.update(measure_peaks(torch))
    if want("ops"):
        extra.update(bench_operators(torch, bard))
    if want("sweep"):
        extra.update(bench_sweep(torch, bard, m, tree, bpe))
    if want("specialized"):
        extra.update(bench_specialized(torch, bard))
    if want("plan"):
        extra.update(bench_plan(torch, bard, args.steps))
    if want("adjoints"):
        extra.update(bench_adjoints(torch, bard, args.steps))
    if want("workspace"):
        extra.update(bench_workspace(torch, bard, args.steps))
    if extra:
        log(f"[bench] extra {extra}")

    # The oracle leg: the FP64 oracle's throughput on a bounded sample (the
    # CPU baseline), the parity of the timed outputs on sampled instances, and
    # the reference torques of the identification experiment.
    cpu = parity = None
    if not args.no_cpu:
        parity = parity_sample(tree, sets)
        log(f"[bench] parity {parity}")
        cpu = cpu_baseline(tree)
        log(f"[bench] cpu baseline {cpu}")
        if want("sysid"):
            extra.update(bench_sysid(torch, bard, sysid_reference()))
            log(f"[bench] sysid {dict((k, v) for k, v in extra.items() if k.startswith('sysid'))}")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "humanoid tree: free root + 3-DOF waist + 1-DOF neck + two 7-DOF arms + "
                               "two 6-DOF legs (31 bodies, nq 37, nv 36, depth 9), 4 end effectors; "
                               "fused RNEA+CRBA+Jacobian through bard_chain after bard_chain_autotune, eager "
                               "C-ABI launches, fresh inputs every step",
                   "batch": B, "tree": "humanoid_large", "rotating_sets": nsets,
                   "bytes_per_eval": bpe, "kernel": kernel},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_if_current(spec_sha),
                     "kernel": kernel, "kernel_avg_us": kavg * 1e3},
        "cpu_baseline": cpu,
        "parity": parity,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
