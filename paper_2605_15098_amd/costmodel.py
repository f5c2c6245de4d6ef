"""Learned schedule selection: data collection, training and evaluation of
the cost model that sv_tune(SV_TUNER_LEARNED) consults.

The model predicts the log of a schedule's device time from host-side
planning features (sv_features) of the (circuit, candidate) pair; the tuner
picks the candidate with the smallest prediction. Training data are device
times measured exactly as the exhaustive tuner measures them
(sv_tune_time). The network's forward pass, gradient and Adam update run in
the library's kernels (sv_mlp_*); this module only moves arrays.

    python -m paper_2605_15098_amd.costmodel collect --circuits 0:600 --per-circuit 6 --out data.npz
    python -m paper_2605_15098_amd.costmodel train --data data.npz --out model.npz
    python -m paper_2605_15098_amd.costmodel eval --model model.npz --circuits 0:50 --out eval.json

Every pass kernel a candidate needs is compiled at run time (about a second
per pass), so `collect` and `eval` compile in a pool of worker processes that
never touch the GPU, started before this process does, while this process
times the circuits already compiled; the library's on-disk module cache
(SV_JIT_CACHE_DIR, default under the temp directory) carries the modules
from the pool to the timed process.
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time
from typing import List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(HERE))
    __package__ = "paper_2605_15098_amd"

from . import sv  # noqa: E402
from . import workloads as W  # noqa: E402

MODEL_PATH = os.path.join(HERE, "cost_model_c64.npz")
IN = sv.SV_FEATURES
LR, BETA1, BETA2, EPS = 1e-3, 0.9, 0.999, 1e-8


def log(msg: str) -> None:
    print(f"[costmodel] {msg}", flush=True)


# ---------------------------------------------------------------- features

def candidate_features(n: int, dtype: str, gates) -> Tuple[list, np.ndarray]:
    cands = sv.sv_tune_candidates(n, dtype)
    X = np.stack([sv.sv_features(n, dtype, gates, c) for c in cands])
    return cands, X


def fit_norm(X: np.ndarray) -> np.ndarray:
    """{mean, 1/std} per feature; constant features get 1/std = 1."""
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    inv = np.where(std > 1e-6, 1.0 / np.maximum(std, 1e-6), 1.0)
    return np.concatenate([mean, inv]).astype(np.float32)


# ---------------------------------------------------------------- ahead-of-time compilation

def _precompile_job(job):
    n, dtype, kind, idx, cand_fields = job
    gates = circuit(kind, idx)[1]
    s = sv.sv_schedule(*cand_fields)
    t0 = time.perf_counter()
    sv.sv_jit_precompile(n, dtype, gates, s)
    return time.perf_counter() - t0


def use_jit_cache() -> str:
    import tempfile
    d = os.environ.setdefault("SV_JIT_CACHE_DIR", os.path.join(tempfile.gettempdir(), "svmi_jit_cache"))
    os.makedirs(d, exist_ok=True)
    return d


def precompile(jobs: Sequence[tuple], workers: int) -> List[float]:
    """Compile every (n, dtype, circuit kind, index, schedule fields) job in a
    pool of processes that only run the compiler. Must run before this
    process first touches the GPU. Returns the compile seconds per job."""
    use_jit_cache()
    if workers <= 1 or len(jobs) <= 1:
        return [_precompile_job(j) for j in jobs]
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        out = []
        for k, t in enumerate(pool.imap(_precompile_job, jobs, chunksize=1)):
            out.append(t)
            if (k + 1) % 50 == 0 or k + 1 == len(jobs):
                log(f"precompiled {k + 1}/{len(jobs)}")
        return out


def _compile_worker(inq, outq) -> None:
    while True:
        item = inq.get()
        if item is None:
            return
        k, job = item
        try:
            t = _precompile_job(job)
        except Exception as e:  # the timed process compiles it again and reports
            log(f"compile job {k} failed: {e}")
            t = -1.0
        outq.put((k, t))


class Pipeline:
    """Compile jobs in a fixed set of compiler-only processes while this
    process times circuits on the GPU. The workers are started before this
    process first touches the GPU and are never restarted (a worker that
    dies ends the run with an error instead); results are handed out in job
    order."""

    def __init__(self, jobs: Sequence[tuple], workers: int):
        import queue as _queue

        self._empty = _queue.Empty
        use_jit_cache()
        self.jobs = list(jobs)
        self.procs = []
        self.results = {}
        self.next = 0
        if workers > 1 and len(self.jobs) > 1:
            ctx = mp.get_context("spawn")
            self.inq, self.outq = ctx.Queue(), ctx.Queue()
            for k, j in enumerate(self.jobs):
                self.inq.put((k, j))
            for _ in range(workers):
                self.inq.put(None)
            self.procs = [ctx.Process(target=_compile_worker, args=(self.inq, self.outq), daemon=True)
                          for _ in range(workers)]
            for p in self.procs:
                p.start()

    def take(self, count: int) -> List[float]:
        """Wait for the next `count` jobs; their compile seconds."""
        out = []
        for _ in range(count):
            k = self.next
            if not self.procs:
                self.results[k] = _precompile_job(self.jobs[k])
            while k not in self.results:
                try:
                    kk, t = self.outq.get(timeout=30)
                    self.results[kk] = t
                except self._empty:
                    if not any(p.is_alive() for p in self.procs):
                        raise RuntimeError("compile workers ended before every job was done")
            out.append(self.results.pop(k))
            self.next += 1
        return out

    def close(self) -> None:
        if self.procs:
            # jobs left in the queue are dropped: without this the process
            # would wait at exit for the queue to hand them to workers that
            # are gone
            self.inq.cancel_join_thread()
            self.outq.cancel_join_thread()
        for p in self.procs:
            if p.is_alive():
                p.terminate()
        for p in self.procs:
            p.join(timeout=5)
        self.procs = []


def circuit(kind: str, idx: int):
    """'train' (20-26 qubits), 'train:lo:hi' (lo..hi qubits) or 'eval'."""
    if kind == "train":
        return W.circuit_random_train(idx)
    if kind.startswith("train:"):
        _, lo, hi = kind.split(":")
        return W.circuit_random_train(idx, lo=int(lo), hi=int(hi))
    if kind == "eval":
        return W.circuit_random_eval(idx)
    raise ValueError(kind)


def _fields(s) -> tuple:
    return tuple(int(getattr(s, name)) for name, _ in sv.sv_schedule._fields_)


# ---------------------------------------------------------------- data collection

def sampled_candidates(n: int, dtype: str, idx: int, per_circuit: int) -> list:
    """All tuner candidates, or a seeded subset of per_circuit of them: the
    regression target is one (circuit, candidate) time, so a subset per
    circuit trades candidates for circuit diversity at the same compile cost."""
    cands = sv.sv_tune_candidates(n, dtype)
    if per_circuit <= 0 or per_circuit >= len(cands):
        return cands
    pick = np.random.default_rng([77, idx]).choice(len(cands), size=per_circuit, replace=False)
    return [cands[int(j)] for j in sorted(pick)]


def collect(idxs: Sequence[int], dtype: str = "c64", repeats: int = 3, workers: int = 12,
            kind: str = "train", per_circuit: int = 0, budget_s: float = 0.0,
            out: Optional[str] = None) -> dict:
    """Time (circuit, candidate) pairs. Stops starting new circuits after
    budget_s seconds (0: no limit) and rewrites `out` every 25 circuits, so a
    run that is cut short keeps what it measured."""
    t_start = time.perf_counter()
    plan = []
    jobs = []
    for i in idxs:
        n, g = circuit(kind, i)
        cands = sampled_candidates(n, dtype, i, per_circuit)
        plan.append((i, n, cands))
        jobs += [(n, dtype, kind, i, _fields(c)) for c in cands]
    log(f"{len(idxs)} circuits, {len(jobs)} (circuit, candidate) pairs")
    pipe = Pipeline(jobs, workers)
    rows, ys, cid, cidx, csec_all, cms_all = [], [], [], [], [], []
    allc = {}

    def pack():
        return {"X": np.concatenate(rows).astype(np.float32) if rows else np.zeros((0, IN), np.float32),
                "ms": np.asarray(ys), "circuit": np.asarray(cid), "cand": np.asarray(cidx),
                "compile_s_pool": np.asarray(csec_all), "compile_ms_timed_process": np.asarray(cms_all)}

    try:
        for k, (i, n, cands) in enumerate(plan):
            if budget_s and time.perf_counter() - t_start > budget_s:
                log(f"time budget reached after {k} circuits")
                break
            csec_all += pipe.take(len(cands))
            g = circuit(kind, i)[1]
            if n not in allc:
                allc[n] = [_fields(c) for c in sv.sv_tune_candidates(n, dtype)]
            X = np.stack([sv.sv_features(n, dtype, g, c) for c in cands])
            st = sv.StateVector(n, dtype)
            ms, cms = sv.sv_tune_time(st.h, g, cands, repeats)
            st.close()
            rows.append(X)
            ys += ms
            cid += [i] * len(cands)
            cidx += [allc[n].index(_fields(c)) for c in cands]
            cms_all += cms
            log(f"timed {k + 1}/{len(plan)}: circuit {i} n={n} best {min(ms):.3f} ms, worst {max(ms):.3f} ms, "
                f"elapsed {time.perf_counter() - t_start:.0f} s")
            if out and (k + 1) % 25 == 0:
                np.savez(out, **pack())
    finally:
        pipe.close()
    d = pack()
    if out:
        np.savez(out, **d)
    return d


# ---------------------------------------------------------------- training (k7 kernels)

def train(X: np.ndarray, ms: np.ndarray, epochs: int = 400, batch: int = 128, seed: int = 0,
          lr: float = LR) -> Tuple[np.ndarray, np.ndarray, list]:
    """Fit the network to log(ms) with MSE and Adam; returns (params, norm,
    per-epoch mean training loss). Runs on the current CUDA device."""
    import torch

    dev = torch.device("cuda")
    norm = fit_norm(X)
    y = np.log(np.asarray(ms, dtype=np.float64)).astype(np.float32)
    P = sv.sv_mlp_param_count(IN)
    params = torch.tensor(W.mlp_init_params(IN, seed).astype(np.float32), device=dev)
    m = torch.zeros(P, device=dev)
    v = torch.zeros(P, device=dev)
    grad = torch.zeros(P, device=dev)
    nrm = torch.tensor(norm, device=dev)
    ws = torch.zeros(sv.sv_mlp_workspace_bytes(IN, batch) // 4, device=dev)
    losses = torch.zeros(1 << 16, device=dev)
    rng = np.random.default_rng(seed)
    N = len(y)
    step = 0
    hist = []
    for ep in range(epochs):
        perm = rng.permutation(N)
        Xd = torch.tensor(np.ascontiguousarray(X[perm]), device=dev)
        yd = torch.tensor(np.ascontiguousarray(y[perm]), device=dev)
        nb = 0
        for s0 in range(0, N, batch):
            b = min(batch, N - s0)
            step += 1
            sv.sv_mlp_grad(params, IN, nrm, Xd[s0:s0 + b], yd[s0:s0 + b], b, grad,
                           losses[nb:nb + 1], ws)
            sv.sv_mlp_adam(params, m, v, grad, P, lr, BETA1, BETA2, EPS, step)
            nb += 1
        hist.append(float(losses[:nb].mean().item()))
        if ep % 50 == 0 or ep + 1 == epochs:
            log(f"epoch {ep}: train mse {hist[-1]:.5f}")
    return params.cpu().numpy(), norm, hist


def predict(params: np.ndarray, norm: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Predicted log ms through the library's forward kernel."""
    import torch

    dev = torch.device("cuda")
    Xd = torch.tensor(np.ascontiguousarray(X, dtype=np.float32), device=dev)
    y = torch.zeros(len(X), device=dev)
    sv.sv_mlp_forward(torch.tensor(params, device=dev), IN, torch.tensor(norm, device=dev), Xd, len(X), y)
    return y.cpu().numpy()


def save(path: str, params: np.ndarray, norm: np.ndarray, meta: dict) -> None:
    np.savez(path, params=params.astype(np.float32), norm=norm.astype(np.float32),
             meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))


def load(path: str = MODEL_PATH):
    with np.load(path, allow_pickle=False) as z:
        meta = json.loads(bytes(z["meta"]).decode())
        return z["params"].copy(), z["norm"].copy(), meta


def install(path: str = MODEL_PATH) -> dict:
    params, norm, meta = load(path)
    sv.sv_set_cost_model(params, IN, norm)
    return meta


# ---------------------------------------------------------------- evaluation

def release() -> None:
    """Return freed state buffers to the device before the next allocation."""
    import torch
    torch.cuda.empty_cache()


def learned_pick(n: int, dtype: str, gates, model_path: str, h) -> Tuple[int, float]:
    """Index (in sv_tune_candidates order) of the model's pick and the
    seconds sv_tune took to make it."""
    install(model_path)
    t1 = time.perf_counter()
    pick = sv.sv_tune(h, gates, sv.SV_TUNER_LEARNED)
    dt = time.perf_counter() - t1
    return [_fields(c) for c in sv.sv_tune_candidates(n, dtype)].index(_fields(pick)), dt


def evaluate(idxs: Sequence[int], model_paths: Sequence[str], dtype: str = "c64", repeats: int = 1,
             workers: int = 12, paper_l: int = 13, budget_s: float = 0.0) -> dict:
    """Per held-out circuit: the time of every candidate (median of `repeats`
    after a warm-up), the pick of each model and its regret against the
    exhaustive best, the untuned default schedule and the paper's schedule
    (LRU victim, data-moving SWAP, l = paper_l; one run, no warm-up)."""
    t_start = time.perf_counter()
    jobs, plan = [], []
    # the untuned default schedule, with the dtype's defaults written out
    # (block, register and pinned qubits) so that it matches its candidate
    default = sv.schedule(block_qubits=14 if dtype == "c64" else 13, reg_qubits=5 if dtype == "c64" else 4,
                          pin_qubits=5 if dtype == "c64" else 3)
    for i in idxs:
        n, g = circuit("eval", i)
        cands = sv.sv_tune_candidates(n, dtype)
        extra = [sv.paper_schedule(paper_l)]
        if _fields(default) not in [_fields(c) for c in cands]:
            extra.append(default)
        plan.append((i, n, cands, extra))
        jobs += [(n, dtype, "eval", i, _fields(c)) for c in cands + extra]
    pipe = Pipeline(jobs, workers)
    per = []
    try:
        for k, (i, n, cands, extra) in enumerate(plan):
            if budget_s and time.perf_counter() - t_start > budget_s:
                log(f"time budget reached after {k} circuits")
                break
            csec = pipe.take(len(cands) + len(extra))
            g = circuit("eval", i)[1]
            st = sv.StateVector(n, dtype)
            picks = {}
            for mp_ in model_paths:
                picks[os.path.basename(mp_)] = learned_pick(n, dtype, g, mp_, st.h)
            try:
                ms = []
                for j, c in enumerate(cands):
                    ms += sv.sv_tune_time(st.h, g, [c], repeats)[0]
                log(f"eval {i} n={n}: {len(cands)} candidates timed, elapsed {time.perf_counter() - t_start:.0f} s")
                pms = sv.sv_tune_time(st.h, g, [sv.paper_schedule(paper_l)], 1)[0][0]
                dfi = [_fields(c) for c in cands].index(_fields(default)) if len(extra) == 1 else -1
                dms = ms[dfi] if dfi >= 0 else sv.sv_tune_time(st.h, g, [default], repeats)[0][0]
            except sv.SvError as e:
                st.close()
                release()
                if e.status != sv.SV_ERR_OUT_OF_MEMORY:
                    raise
                log(f"eval {i} n={n}: not measured ({e.message})")
                per.append({"circuit": i, "n": n, "not_measured": e.message})
                continue
            st.close()
            release()
            best = int(np.argmin(ms))
            rec = {"circuit": i, "n": n, "ms": ms, "best": best, "default_ms": dms, "paper_ms": pms,
                   "cold_compile_s": float(sum(csec[:len(cands)])), "models": {}}
            for name, (li, tune_s) in picks.items():
                rec["models"][name] = {"pick": li, "ms": ms[li], "regret": ms[li] / ms[best] - 1.0,
                                       "gain_vs_default": dms / ms[li], "gain_vs_paper": pms / ms[li],
                                       "tune_s": tune_s}
            per.append(rec)
            log(f"eval {i} n={n}: best {ms[best]:.1f} ms, default {dms:.1f} ms, paper {pms:.1f} ms; " +
                ", ".join(f"{nm} {r['ms']:.1f} ms ({100 * r['regret']:.1f}%)" for nm, r in rec["models"].items()))
    finally:
        pipe.close()
    done = [r for r in per if "ms" in r]
    summary = {}
    for mp_ in model_paths:
        name = os.path.basename(mp_)
        reg = np.array([r["models"][name]["regret"] for r in done])
        summary[name] = {
            "meta": load(mp_)[2], "measured": len(done),
            "regret_median": float(np.median(reg)) if len(reg) else None,
            "regret_p90": float(np.percentile(reg, 90)) if len(reg) else None,
            "picked_best": int(sum(r["models"][name]["pick"] == r["best"] for r in done)),
            "gain_vs_default_median": float(np.median([r["models"][name]["gain_vs_default"] for r in done])),
            "gain_vs_paper_median": float(np.median([r["models"][name]["gain_vs_paper"] for r in done]))}
    dreg = np.array([r["default_ms"] / r["ms"][r["best"]] - 1.0 for r in done])
    return {"circuits": per, "models": summary,
            "default_regret_median": float(np.median(dreg)) if len(dreg) else None,
            "default_regret_p90": float(np.percentile(dreg, 90)) if len(dreg) else None}


def _range(spec: str) -> List[int]:
    """'a:b' or a comma-separated list of such ranges and single indices."""
    out = []
    for part in spec.split(","):
        if ":" in part:
            a, b = part.split(":")
            out += list(range(int(a), int(b)))
        else:
            out.append(int(part))
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--circuits", default="0:120")
    c.add_argument("--qubits", default="20:26", help="lo:hi qubits of the training circuits")
    c.add_argument("--per-circuit", type=int, default=0, help="candidates timed per circuit (0: all)")
    c.add_argument("--budget", type=float, default=0.0, help="seconds after which no new circuit starts")
    c.add_argument("--workers", type=int, default=12)
    c.add_argument("--out", required=True)
    t = sub.add_parser("train")
    t.add_argument("--data", required=True, help="one or more collected .npz files, comma separated")
    t.add_argument("--epochs", type=int, default=400)
    t.add_argument("--out", required=True)
    e = sub.add_parser("eval")
    e.add_argument("--model", default=MODEL_PATH, help="one or more model files, comma separated")
    e.add_argument("--circuits", default="0:50")
    e.add_argument("--repeats", type=int, default=1)
    e.add_argument("--budget", type=float, default=0.0)
    e.add_argument("--workers", type=int, default=12)
    e.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "collect":
        lo, hi = a.qubits.split(":")
        kind = "train" if (lo, hi) == ("20", "26") else f"train:{lo}:{hi}"
        d = collect(_range(a.circuits), workers=a.workers, kind=kind, per_circuit=a.per_circuit,
                    budget_s=a.budget, out=a.out)
        log(f"wrote {a.out}: {len(d['ms'])} timings of {len(set(d['circuit'].tolist()))} circuits")
    elif a.cmd == "train":
        Xs, mss, cids = [], [], []
        for k, path in enumerate(a.data.split(",")):
            with np.load(path, allow_pickle=False) as z:
                Xs.append(z["X"])
                mss.append(z["ms"])
                cids.append(z["circuit"] + 100000 * k)
        X, ms, cid = np.concatenate(Xs), np.concatenate(mss), np.concatenate(cids)
        params, norm, hist = train(X, ms, epochs=a.epochs)
        pred = predict(params, norm, X)
        meta = {"features": sv.FEATURE_NAMES, "samples": int(len(ms)),
                "circuits": int(len(set(cid.tolist()))), "epochs": a.epochs, "lr": LR,
                "data": [os.path.basename(p) for p in a.data.split(",")],
                "n_range": [int(X[:, 0].min()), int(X[:, 0].max())],
                "final_train_mse": hist[-1],
                "train_mse_check": float(np.mean((pred - np.log(ms)) ** 2))}
        save(a.out, params, norm, meta)
        log(f"wrote {a.out}: {meta}")
    else:
        res = evaluate(_range(a.circuits), a.model.split(","), repeats=a.repeats, workers=a.workers,
                       budget_s=a.budget)
        with open(a.out, "w") as fh:
            json.dump(res, fh, indent=1)
        for name, m in res["models"].items():
            log(f"{name}: regret median {m['regret_median']}, p90 {m['regret_p90']}, "
                f"picked best {m['picked_best']}/{m['measured']}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
