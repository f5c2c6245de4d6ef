"""Benchmark: 32-qubit QPE on one MI355X, complex64, partitioned schedule.

One step = one sv_apply_circuit of the whole 32-qubit QPE gate list (559
gates + 15 SWAP relabels) on a 2^32-amplitude complex64 state that is
already resident in HBM. The JSON line reports gate-sweeps/s (gates / step
time), effective HBM GB/s (algorithmic bytes of the passes / step time), the
roofline of the block-pass kernel measured with HIP events on its stream, the
plain complex128 path and the other schedules on the same GPU, each with its
error against the FP64 QPE closed form over the whole state, and the oracle
on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
    python bench.py --cpu-full      # CPU oracle only: whole circuits, median of 3
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "gate-sweeps/s + effective HBM GB/s (% roofline), 28-32q QPE, c64 vs c128"
HBM_PEAK_GBPS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    # the sources the run-time compiled block-pass kernels are generated from
    for f in ("k2_device.h", "k2_abi.h", "jit.cpp", "plan.cpp", "plan.h"):
        with open(os.path.join(ROOT, "paper_2605_15098_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source; else None."""
    path = os.path.join(PROFILES, "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    rec = data.get(f"{kernel}:{workload}")
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def time_apply(sim, gates, sched, steps, warmup, kernel_timing=False):
    import torch
    from paper_2605_15098_amd import sv

    sv.sv_set_kernel_timing(sim.h, kernel_timing)
    # block passes are compiled for their op lists once, ahead of timing; the
    # circuit's SWAP relabels alternate between two layouts, so two calls' worth
    sv.sv_prepare(sim.h, gates, sched, 2)
    for _ in range(warmup):
        sim.apply(gates, sched)
    torch.cuda.synchronize()
    kms = [0.0, 0.0, 0.0]
    kl = [0, 0, 0]
    dev_ms = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        sim.apply(gates, sched)
        st = sim.stats()  # waits for this step's last event
        dev_ms += st["device_ms"]
        for k in range(3):
            kms[k] += st["kernel_ms"][k]
            kl[k] += st["kernel_launches"][k]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sv.sv_set_kernel_timing(sim.h, False)
    return wall, dev_ms, kms, kl, st


class Reference:
    """The FP64 QPE closed form (oracle), evaluated once per (n, phi) into
    host memory when it fits, else chunk by chunk per comparison."""

    def __init__(self, n, phi):
        from oracle import timing as T

        self.n, self.phi = n, phi
        need = 16 << (n - 1)
        self.cache = {} if T.mem_available() > 3 * need + (16 << 30) else None

    def check(self, sim, gates, sched):
        """Apply the circuit once from |0...0> and compare every amplitude."""
        from oracle import compare as C
        from oracle import qpe as cf
        from paper_2605_15098_amd import sv

        sim.reset()
        sim.apply(gates, sched)
        n, t = self.n, self.n - 1
        m, _, pmax = sim.qpe_readout()
        t0 = time.perf_counter()
        ref = C.qpe_reference(n, self.phi, self.cache)
        err = C.stream_errors(lambda o, c: sv.sv_state_range(sim.h, o, c, sim.dtype), 1 << n, ref,
                              chunk=1 << 23)
        out = {"argmax": int(m), "argmax_expected": cf.qpe_argmax(t, self.phi), "p_max": pmax,
               "max_abs_err": err["max_abs"], "max_abs_err_component": err["max_abs_component"],
               "one_minus_fidelity": err["one_minus_fidelity"], "norm_err": err["norm_err"],
               "amplitudes_compared": 1 << n, "reference": "FP64 QPE closed form (oracle)",
               "check_s": round(time.perf_counter() - t0, 1)}
        return out

    def drop(self):
        self.cache = None


def roofline(kms, kl, pass_bytes, name, workload, kernel):
    achieved = (kl * pass_bytes) / (kms / 1000.0) / 1e9 if kl else 0.0
    return {"kernel": name, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS, "traffic": measured_traffic(kernel, workload),
            "algorithmic_bytes_per_launch": pass_bytes, "launches": kl,
            "avg_launch_ms": kms / kl if kl else None}


def hbm_reference(n, ab, block, pin, reg, reps=5):
    """Measured ceilings on this GPU for the block pass's traffic: a plain
    streaming copy and an in-place rewrite (sv_stream_probe) over buffers of
    the state's size, and the block-pass kernel itself on a one-gate circuit
    (Z on qubit 0: one pass whose only work is one phase multiply per
    amplitude), all timed with HIP events on the current stream."""
    import torch
    from paper_2605_15098_amd import sv
    from paper_2605_15098_amd import workloads as W

    out = {}
    nbytes = ab << n

    def timed(fn):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        fn()
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            ev[0].record()
            fn()
            ev[1].record()
            ev[1].synchronize()
            ms.append(ev[0].elapsed_time(ev[1]))
        return float(np.median(ms))

    half = nbytes // 2
    buf = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    a, b = buf[: half // 4], buf[half // 4:]
    ms = timed(lambda: sv.sv_stream_probe(b, a, half, 0))
    out["stream_copy"] = {"bytes": 2 * half, "ms": ms, "GBps": 2 * half / ms / 1e6,
                          "what": f"copy of {half >> 30} GiB to another {half >> 30} GiB"}
    ms = timed(lambda: sv.sv_stream_probe(buf, None, nbytes, 1))
    out["stream_in_place"] = {"bytes": 2 * nbytes, "ms": ms, "GBps": 2 * nbytes / ms / 1e6,
                              "what": f"read and rewrite of {nbytes >> 30} GiB in place"}
    del buf, a, b
    torch.cuda.empty_cache()
    sim = sv.StateVector(n, "c64" if ab == 8 else "c128")
    g = W.gates_from_tuples([("Z", 0, -1, 0.0)])
    sched = sv.schedule(block_qubits=block, pin_qubits=pin, reg_qubits=reg)
    sv.sv_prepare(sim.h, g, sched, 1)

    def one():
        sim.apply(g, sched)
    ms = timed(one)
    st = sim.stats()
    out["block_pass_one_gate"] = {"bytes": 2 * nbytes, "ms": ms, "GBps": 2 * nbytes / ms / 1e6,
                                  "passes": st["passes"],
                                  "what": "the block-pass kernel on a one-gate circuit (Z on qubit 0), "
                                          "same block size, pins and register tile"}
    sim.close()
    torch.cuda.empty_cache()
    return out


def cpu_baseline(n, phi, budget_s=20.0):
    """The oracle on this host's cores on a bounded sample of the same
    workload: its float build (the precision of the complex64 path) applies
    a strided sample of the 32-qubit QPE's non-SWAP gates, in circuit order,
    to a 2^n state in one call (gate loop only; the state is allocated and
    first-touched by the oracle's threads beforehand)."""
    from oracle import timing as T
    from paper_2605_15098_amd import workloads as W

    while n > 20 and (8 << n) + (8 << 30) > T.mem_available():
        n -= 1
    gates = W.qpe_gates(n, phi)
    body = gates[gates["op"] != 9]
    S = T.alloc_state(n, "f32")
    T.time_gate_loop(n, body[1:2], S, "f32")  # starts the oracle's threads
    probe = T.time_gate_loop(n, body[1:3], S, "f32") / 2  # Hadamard-layer gates
    k = max(1, min(len(body), int(budget_s / max(probe, 1e-6))))
    stride = max(1, len(body) // k)
    sample = body[::stride][:k]
    el = T.time_gate_loop(n, sample, S, "f32")
    del S
    kinds = {int(o): int(np.sum(sample["op"] == o)) for o in np.unique(sample["op"])}
    return {"value": len(sample) / el, "unit": "gate-sweeps/s", "cores": T.num_threads("f32"), "kind": "oracle",
            "sample": f"{'every' if stride == 1 else f'every {stride}-th'} non-SWAP gate of the {n}-qubit QPE "
                      f"circuit ({len(sample)} gates: "
                      f"{kinds.get(7, 0)} controlled phases, {kinds.get(0, 0)} Hadamards, {kinds.get(1, 0)} X) in "
                      f"circuit order, applied by the oracle's float build (complex64 state, the precision of "
                      f"the GPU value) in one call on the 2^{n} state, gate loop only: {el:.1f} s",
            "host": T.host_info()}


def cpu_full():
    """Whole-circuit timings of the oracle on the host: the 28-qubit QPE in
    FP64 and in the float build, median of 3 with 2-s pauses (as the paper
    times its runs, Section IV-B), and the 24-qubit QPE in FP64 on all threads
    and on one thread (the scaling reference)."""
    from oracle import timing as T
    from paper_2605_15098_amd import workloads as W

    out = {"host": T.host_info(), "runs": []}
    for n, prec, threads in ((28, "f64", None), (28, "f32", None), (24, "f64", None), (24, "f64", 1)):
        if (16 if prec == "f64" else 8) << n > T.mem_available() - (8 << 30):
            out["runs"].append({"n": n, "precision": prec, "status": "not measured (host memory)"})
            continue
        phi = W.phi_for_seed(n)
        gates = W.qpe_gates(n, phi)
        G = W.qpe_gate_count(n)[0]
        nthr = T.num_threads(prec)
        if threads:
            T.set_threads(threads, prec)
        log(f"cpu-full n={n} {prec} threads={threads or nthr}")
        med, times = T.median_of_runs(n, gates, prec)
        if threads:
            T.set_threads(nthr, prec)
        rec = {"n": n, "precision": prec, "threads": threads or nthr, "gates": G, "median_s": med,
               "times_s": times, "gate_sweeps_per_s": G / med,
               "what": "whole QPE circuit (SWAPs included, as data moves), gate loop only, median of 3, "
                       "2-s pauses"}
        log(f"  {rec}")
        out["runs"].append(rec)
    return out


SWEEP_NS = (4, 8, 12, 16, 20, 22, 24, 26, 28, 30, 32, 34)


def sweep_configs(n):
    """The paper's experiment (Section IV-B) on this GPU: the unpartitioned
    per-gate sweep (the paper's baseline), the paper's partitioning (LRU
    victim, data-moving SWAP) over block sizes, the dependence-graph schedule
    (the library default), and for n >= 28 the Infinity Cache outer tier."""
    from paper_2605_15098_amd import sv

    out = [("plain", "plain", sv.schedule("plain"))]
    for l in sorted({min(n - 1, x) for x in (6, 8, 10, 12, 13, 14)}):
        if l >= 2:
            out.append((f"paper-lru-l{l}", "paper-lru", sv.paper_schedule(l)))
    out.append(("graph-default", "graph", sv.schedule()))
    if n >= 28:
        for l2 in (22, 24, 26):
            out.append((f"graph-outer-l2-{l2}", "graph-outer", sv.schedule(outer_qubits=l2)))
    return out


def sweep_gates(n):
    import math
    from paper_2605_15098_amd import workloads as W

    # the paper's U(n): phi = 2^-t, read as counting value 1 with probability 1
    return W.qpe_gates(n, math.ldexp(1.0, -(n - 1)))


def sweep_precompile(cache_dir, workers=8):
    """Compile every sweep configuration's passes into cache_dir (CPU only)."""
    from concurrent.futures import ProcessPoolExecutor

    os.makedirs(cache_dir, exist_ok=True)
    jobs = [(n, name) for n in SWEEP_NS for name, _, _ in sweep_configs(n)]
    with ProcessPoolExecutor(workers) as pool:
        list(pool.map(_precompile_one, [(cache_dir, n, name) for n, name in jobs]))
    return len(jobs)


def _precompile_one(args):
    cache_dir, n, name = args
    os.environ["SV_JIT_CACHE_DIR"] = cache_dir
    from paper_2605_15098_amd import sv

    sched = dict((nm, sc) for nm, _, sc in sweep_configs(n))[name]
    if sched.mode == 1:
        sv.sv_jit_precompile(n, "c64", sweep_gates(n), sched)


def sweep(reps=2):
    """Time every configuration of sweep_configs at every n (complex64, the
    paper's precision): device ms of one circuit from |0...0> (median of
    `reps` after one warm-up), passes, SWAPs, algorithmic GB/s, and the
    readout check (counting value 1 with probability ~1); beside it the
    oracle's float build on the host (whole circuit up to 24 qubits, a
    strided sample of the circuit above) for the GPU/CPU speedup."""
    import torch
    from oracle import timing as T
    from paper_2605_15098_amd import sv
    from paper_2605_15098_amd import workloads as W

    rows = []
    for n in SWEEP_NS:
        gates = sweep_gates(n)
        G = W.qpe_gate_count(n)[0]
        sim = sv.StateVector(n, "c64")
        for name, family, sched in sweep_configs(n):
            ms = []
            for r in range(reps + 1):
                sim.reset()
                sim.apply(gates, sched)
                st = sim.stats()
                if r:
                    ms.append(st["device_ms"])
            m, _, pmax = sim.qpe_readout()
            dms = float(np.median(ms))
            row = {"n": n, "config": name, "family": family, "l": st["block_qubits"],
                   "outer_qubits": int(sched.outer_qubits), "device_ms": dms, "passes": st["passes"],
                   "swaps": st["swaps"], "phases": st["phases"], "gate_sweeps_per_s": G / (dms / 1e3),
                   "effective_GBps": st["bytes"] / (dms / 1e3) / 1e9, "argmax": m, "p_max": pmax}
            assert m == 1 and abs(pmax - 1.0) < 1e-4, (n, name, m, pmax)
            rows.append(row)
            log(f"sweep n={n} {name}: {dms:.3f} ms, {st['passes']} passes, {st['swaps']} swaps, "
                f"{row['effective_GBps']:.0f} GB/s")
        sim.close()
        torch.cuda.empty_cache()
    cpu = []
    for n in SWEEP_NS:
        if n > 32 or (8 << n) + (8 << 30) > T.mem_available():
            continue
        gates = sweep_gates(n)
        body = gates[gates["op"] != 9]
        S = T.alloc_state(n, "f32")
        if n <= 24:
            el = T.time_gate_loop(n, gates, S, "f32")
            rate, what = len(body) / el, "whole circuit (SWAPs as data moves)"
        else:
            T.time_gate_loop(n, body[1:2], S, "f32")
            probe = T.time_gate_loop(n, body[1:3], S, "f32") / 2
            k = max(4, min(len(body), int(4.0 / max(probe, 1e-6))))
            stride = max(1, len(body) // k)
            sample = body[::stride][:k]
            el = T.time_gate_loop(n, sample, S, "f32")
            rate, what = len(sample) / el, f"every {stride}-th non-SWAP gate ({len(sample)} gates)"
        del S
        cpu.append({"n": n, "gate_sweeps_per_s": rate, "what": what})
        log(f"sweep cpu n={n}: {rate:.2f} gate-sweeps/s ({what})")
    return {"gpu": rows, "cpu_oracle_f32": cpu, "host": T.host_info()}


def bench_batch(steps):
    """256 QPE instances (12..22 qubits, complex64) in one persistent launch
    under a captured graph, schedule picked by the batch autotuner."""
    import torch
    from oracle import compare as C
    from oracle import qpe as cf
    from paper_2605_15098_amd import sv
    from paper_2605_15098_amd import workloads as W

    inst = W.batch_instances(256, seed=4)
    gl = [W.qpe_gates(n, p) for n, p in inst]
    states = [sv.StateVector(n, "c64") for n, _ in inst]
    hs = [s.h for s in states]
    t0 = time.perf_counter()
    best = sv.sv_tune_batch(hs, gl)
    tune_s = time.perf_counter() - t0
    log(f"batch tuner: block_qubits={best.block_qubits} fuse_k={best.fuse_k} ({tune_s:.1f} s)")
    for _ in range(2):
        sv.sv_apply_batch(hs, gl, best)
    torch.cuda.synchronize()
    dev = []
    t0 = time.perf_counter()
    for _ in range(steps):
        sv.sv_apply_batch(hs, gl, best)
        dev.append(states[0].stats()["device_ms"])
    wall = (time.perf_counter() - t0) / steps
    alg_bytes = float(sum(s.stats()["bytes"] for s in states))
    # correctness: every instance from |0>, every amplitude against the closed form
    for s in states:
        s.reset()
    sv.sv_apply_batch(hs, gl, best)
    worst, worst_fid, argmax_ok = 0.0, 0.0, 0
    for s, (n, p) in zip(states, inst):
        t = n - 1
        m, _, _ = s.qpe_readout()
        argmax_ok += int(m == cf.qpe_argmax(t, p))
        e = C.stream_errors(lambda o, c, s=s: sv.sv_state_range(s.h, o, c, "c64"), 1 << n,
                            C.qpe_reference(n, p), chunk=1 << 22, threads=4)
        worst = max(worst, e["max_abs"])
        worst_fid = max(worst_fid, e["one_minus_fidelity"])
    for s in states:
        s.close()
    torch.cuda.empty_cache()
    dms = float(np.median(dev))
    res = {"instances": len(inst), "qubits": [min(n for n, _ in inst), max(n for n, _ in inst)],
           "instances_per_s": len(inst) / wall, "ms_per_batch": 1000 * wall,
           "device_ms_per_batch": dms, "schedule": {"block_qubits": best.block_qubits, "fuse_k": best.fuse_k},
           "algorithmic_bytes_per_batch": alg_bytes,
           "effective_GBps_device": alg_bytes / (dms / 1000.0) / 1e9 if dms > 0 else None,
           "hbm_frac_device": alg_bytes / (dms / 1000.0) / 1e9 / HBM_PEAK_GBPS if dms > 0 else None,
           "tuning_s": tune_s, "max_abs_err_worst_instance": worst, "one_minus_fidelity_worst": worst_fid,
           "argmax_exact": f"{argmax_ok}/{len(inst)}", "amplitudes_compared": "all"}
    log(f"batch: {res}")
    return res


def bench_dense_fusion(steps, n=28, cases=(("blocked-depth24", 24),)):
    """Matrix-core windows where the circuit is dense: circuits that keep
    `depth` layers of RX and RY on every qubit with CZ along 5-qubit groups
    before coupling the groups (two rounds; workloads.blocked_dense_circuit),
    or, for depth 0, layers of rotations with CNOT ladders over all qubits
    (about ten dense gates per window: the cost gate admits none). fuse_k 5
    (windows through the matrix cores where the measured cost gate admits
    them) against fuse_k 1, in both precisions: device time per circuit,
    passes, gates taken into windows, and the largest amplitude difference
    between the fused and unfused final states (both from |0>)."""
    import torch
    from paper_2605_15098_amd import sv
    from paper_2605_15098_amd import workloads as W

    res = {"n": n}
    for name, depth in cases:
        rng = np.random.default_rng(depth)
        gates = (W.blocked_dense_circuit(n, 2, depth, rng) if depth > 0
                 else W.layered_dense_circuit(n, 4, rng))
        res[name] = {"gates": int(len(gates))}
        for dt in ("c64", "c128"):
            sims, row = {}, {}
            for fuse in (1, 5):
                sched = sv.schedule(fuse_k=fuse)
                s = sv.StateVector(n, dt)
                wall, dms, _, _, st = time_apply(s, gates, sched, steps, 1)
                s.reset()
                s.apply(gates, sched)
                row[f"fuse_k{fuse}"] = {"ms_per_circuit": 1000.0 * wall / steps, "device_ms": dms / steps,
                                        "passes": st["passes"], "gates_in_windows": st["fused"]}
                sims[fuse] = s
            diff = 0.0
            chunk = 1 << 24
            for o in range(0, 1 << n, chunk):
                a = sv.sv_state_range(sims[1].h, o, chunk, dt).astype(np.complex128)
                b = sv.sv_state_range(sims[5].h, o, chunk, dt).astype(np.complex128)
                diff = max(diff, float(np.max(np.abs(a - b))))
            for s in sims.values():
                s.close()
            torch.cuda.empty_cache()
            row["speedup_fused"] = row["fuse_k1"]["ms_per_circuit"] / row["fuse_k5"]["ms_per_circuit"]
            row["max_abs_diff_fused_vs_unfused"] = diff
            res[name][dt] = row
            log(f"dense fusion {name} {dt}: {row}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--dtype", default="c64")
    ap.add_argument("--block", type=int, default=-1, help="block qubits (default: 14 for c64, library default for c128)")
    ap.add_argument("--pin", type=int, default=-1, help="pinned low qubits (default: 5 for c64)")
    ap.add_argument("--reg", type=int, default=-1, help="register qubits per thread (default: 5 for c64)")
    ap.add_argument("--policy", default="graph", choices=("graph", "lookahead", "lru"),
                    help="gate order and block gathering (default: over the dependence graph)")
    ap.add_argument("--quick", action="store_true", help="skip comparison runs, batch and CPU baseline")
    ap.add_argument("--no-check", action="store_true", help="skip the full-state error checks")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-full", action="store_true",
                    help="only time the CPU oracle on whole circuits (median of 3) and print that record")
    ap.add_argument("--sweep", action="store_true",
                    help="only run the paper's experiment: QPE with phi = 2^-t over n and block sizes")
    ap.add_argument("--sweep-precompile", metavar="DIR",
                    help="compile the sweep's passes into DIR on the host and exit (no GPU)")
    ap.add_argument("--only", choices=("batch", "dense-fusion"),
                    help="run only that section (batched QPE or dense-circuit fusion) and print its record")
    ap.add_argument("--dense-depth", type=int, default=-1,
                    help="with --only dense-fusion: only the circuit of this depth (0: layered)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, run one plain 4 GiB read + 4 GiB write kernel "
                         "(the reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    if args.cpu_full:
        print(json.dumps(cpu_full()), flush=True)
        return
    if args.sweep_precompile:
        print(json.dumps({"precompiled": sweep_precompile(args.sweep_precompile)}), flush=True)
        return
    if args.only:
        import torch
        from paper_2605_15098_amd import sv

        sv.load()
        torch.cuda.set_device(0)
        cases = (("layered-depth1", 0), ("blocked-depth8", 8), ("blocked-depth12", 12), ("blocked-depth24", 24))
        if args.dense_depth >= 0:
            cases = tuple(c for c in cases if c[1] == args.dense_depth)
        rec = bench_batch(args.steps) if args.only == "batch" else bench_dense_fusion(args.steps, cases=cases)
        print(json.dumps(rec), flush=True)
        return
    if args.sweep:
        import torch
        from paper_2605_15098_amd import sv

        sv.load()
        torch.cuda.set_device(0)
        print(json.dumps(sweep()), flush=True)
        return

    import torch
    from paper_2605_15098_amd import sv
    from paper_2605_15098_amd import workloads as W

    sv.load()
    torch.cuda.set_device(0)
    n = args.n
    seed = n
    phi = W.phi_for_seed(seed)
    gates = W.qpe_gates(n, phi)
    ngates = W.qpe_gate_count(n)[0]
    ab = 8 if args.dtype == "c64" else 16
    # complex64 default: the schedule the tuner sweep found fastest on this
    # workload (2^14-amplitude blocks, 5 pinned low qubits = 256-byte runs,
    # 32 amplitudes per thread); complex128 keeps the library defaults
    c64 = args.dtype == "c64"
    block = args.block if args.block >= 0 else (14 if c64 else 0)
    pin = args.pin if args.pin >= 0 else (5 if c64 else 0)
    reg = args.reg if args.reg >= 0 else (5 if c64 else 0)
    sched = sv.schedule(block_qubits=block, pin_qubits=pin, reg_qubits=reg, swap_policy=args.policy)
    ref = None if args.no_check else Reference(n, phi)

    log(f"workload qpe n={n} dtype={args.dtype} phi_seed={seed} gates={ngates}")
    sim = sv.StateVector(n, args.dtype)
    wall, dev_ms, kms, kl, st = time_apply(sim, gates, sched, args.steps, args.warmup, kernel_timing=True)
    ms_per_step = 1000.0 * wall / args.steps
    value = ngates / (wall / args.steps)
    eff_gbps = st["bytes"] / (wall / args.steps) / 1e9
    pass_bytes = 2.0 * ab * 2.0 ** n
    rl = roofline(kms[1], kl[1], pass_bytes, "svk2_pass_* (block-resident pass)",
                  f"qpe{n}-{args.dtype}-{args.policy}-l{st['block_qubits']}p{pin}r{reg}", "k2")
    log(f"{ms_per_step:.2f} ms/step, {value:.1f} gate-sweeps/s, {eff_gbps:.0f} GB/s effective, "
        f"k2 {rl['achieved']:.0f} GB/s over {kl[1]} launches")
    check = ref.check(sim, gates, sched) if ref else None
    log(f"parity: {check}")
    sim.close()
    del sim
    torch.cuda.empty_cache()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "gate-sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.dtype == "c64" else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"qpe-{n}q-{'complex64' if args.dtype == 'c64' else 'complex128'}-partitioned",
            "n_qubits": n, "counting_qubits": n - 1, "phi_seed": seed, "phi": phi,
            "gates_per_step": ngates, "swap_relabels": (n - 1) // 2,
            "schedule": {"mode": "partitioned", "block_qubits": st["block_qubits"],
                         "pin_qubits": pin or "default", "reg_qubits": reg or "default",
                         "swap_policy": args.policy, "remap": "virtual", "diag_free": True},
            "passes_per_step": st["passes"], "swaps_per_step": st["swaps"],
        },
        "effective_GBps": eff_gbps,
        "effective_hbm_frac": eff_gbps / HBM_PEAK_GBPS,
        "device_ms_per_step": dev_ms / args.steps,
        "roofline": rl,
        "parity": check,
    }

    out["hbm_reference"] = hbm_reference(n, ab, block, pin, reg)
    log(f"hbm reference: {out['hbm_reference']}")
    if args.copy_calibration:
        # one elementwise kernel that reads 4 GiB and writes 4 GiB: the
        # reference against which HBM byte counters are scaled
        src = torch.ones(1 << 30, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
    if not args.quick:
        comps = {}
        for name, dt, sch, st_, wu in (
                ("c128-plain", "c128", sv.schedule("plain"), 1, 1),
                ("c128-partitioned", "c128", sv.schedule(), 3, 1),
                ("c128-fused-k5", "c128", sv.schedule(fuse_k=5), 2, 1),
                ("c64-fused-k5", "c64", sv.schedule(block_qubits=block, pin_qubits=pin, reg_qubits=reg, fuse_k=5),
                 3, 1),
                ("c64-partitioned-l13-pin4-reg4", "c64", sv.schedule(block_qubits=13, pin_qubits=4, reg_qubits=4),
                 4, 2),
                ("c64-lookahead-circuit-order", "c64",
                 sv.schedule(block_qubits=block, pin_qubits=pin, reg_qubits=reg, swap_policy="lookahead"), 4, 2),
                ("c64-partitioned-outer-tier-l2-25", "c64",
                 sv.schedule(block_qubits=block, pin_qubits=pin, reg_qubits=reg, outer_qubits=25), 4, 2),
                ("c64-plain", "c64", sv.schedule("plain"), 1, 1),
                ("c64-paper-lru-l13", "c64", sv.paper_schedule(13), 1, 1)):
            log(f"comparison {name}")
            s2 = sv.StateVector(n, dt)
            w2, d2, km2, kl2, st2 = time_apply(s2, gates, sch, st_, wu, kernel_timing=(name == "c128-partitioned"))
            comps[name] = {"ms_per_step": 1000.0 * w2 / st_, "gate_sweeps_per_s": ngates / (w2 / st_),
                           "effective_GBps": st2["bytes"] / (w2 / st_) / 1e9, "passes": st2["passes"],
                           "swaps": st2["swaps"], "fused_windows": st2["fused"]}
            if name == "c128-partitioned":
                out["roofline_c128"] = roofline(km2[1], kl2[1], 2.0 * 16 * 2.0 ** n,
                                                "svk2_pass_* (block-resident pass, complex128)",
                                                f"qpe{n}-c128-graph-l{st2['block_qubits']}p0r0", "k2")
            if ref:
                comps[name]["error"] = ref.check(s2, gates, sch)
            log(f"  {comps[name]}")
            s2.close()
            del s2
            torch.cuda.empty_cache()
        out["comparisons"] = comps
        out["speedup_vs_c128_plain"] = value / comps["c128-plain"]["gate_sweeps_per_s"]
    if ref:
        ref.drop()
    if not args.quick:
        out["batch_qpe256"] = bench_batch(args.steps)
        out["dense_fusion"] = bench_dense_fusion(2)
    if not args.quick and not args.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(n, phi)
        log(f"  {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
