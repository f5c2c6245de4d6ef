"""Learned schedule selection: data collection, training and evaluation of
the cost model that sv_tune(SV_TUNER_LEARNED) consults.

The model predicts the log of a schedule's device time from host-side
planning features (sv_features) of the (circuit, candidate) pair; the tuner
picks the candidate with the smallest prediction. Training data are device
times measured exactly as the exhaustive tuner measures them
(sv_tune_time). The network's forward pass, gradient and Adam update run in
the library's kernels (sv_mlp_*); this module only moves arrays.

    python -m paper_2605_15098_amd.costmodel collect --circuits 0:120 --out data.npz
    python -m paper_2605_15098_amd.costmodel train --data data.npz --out model.npz
    python -m paper_2605_15098_amd.costmodel eval --model model.npz --per-n 5 --out eval.json

Every pass kernel a candidate needs is compiled at run time (several seconds
per schedule), so `collect` and `eval` first compile all candidates in a pool
of worker processes that never touch the GPU; the library's on-disk module
cache (SV_JIT_CACHE_DIR, default under the temp directory) then serves the
timed process.
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

def collect(idxs: Sequence[int], dtype: str = "c64", repeats: int = 3, workers: int = 12,
            kind: str = "train") -> dict:
    jobs = []
    for i in idxs:
        n, g = circuit(kind, i)
        for c in sv.sv_tune_candidates(n, dtype):
            jobs.append((n, dtype, kind, i, _fields(c)))
    log(f"{len(idxs)} circuits, {len(jobs)} (circuit, candidate) pairs")
    t0 = time.perf_counter()
    csec = precompile(jobs, workers)
    log(f"compiled in {time.perf_counter() - t0:.1f} s")
    rows, ys, cid, cidx, cms_all = [], [], [], [], []
    for k, i in enumerate(idxs):
        n, g = circuit(kind, i)
        cands, X = candidate_features(n, dtype, g)
        st = sv.StateVector(n, dtype)
        ms, cms = sv.sv_tune_time(st.h, g, cands, repeats)
        st.close()
        rows.append(X)
        ys += ms
        cid += [i] * len(cands)
        cidx += list(range(len(cands)))
        cms_all += cms
        log(f"timed {k + 1}/{len(idxs)}: circuit {i} n={n} best {min(ms):.3f} ms, worst {max(ms):.3f} ms, "
            f"load/compile {sum(cms) / 1e3:.1f} s")
    return {"X": np.concatenate(rows).astype(np.float32), "ms": np.asarray(ys),
            "circuit": np.asarray(cid), "cand": np.asarray(cidx),
            "compile_s_pool": np.asarray(csec), "compile_ms_timed_process": np.asarray(cms_all)}


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


def evaluate(idxs: Sequence[int], model_path: str, dtype: str = "c64", repeats: int = 3,
             workers: int = 12, paper_l: int = 13) -> dict:
    """Per held-out circuit: exhaustive times of every candidate, the learned
    pick, its regret, the paper's default schedule and the tuning costs."""
    jobs = []
    for i in idxs:
        n, g = circuit("eval", i)
        for c in sv.sv_tune_candidates(n, dtype):
            jobs.append((n, dtype, "eval", i, _fields(c)))
        jobs.append((n, dtype, "eval", i, _fields(sv.paper_schedule(paper_l))))
    t0 = time.perf_counter()
    csec = precompile(jobs, workers)
    log(f"compiled {len(jobs)} schedules in {time.perf_counter() - t0:.1f} s")
    meta = install(model_path)
    per = []
    k = 0
    for i in idxs:
        n, g = circuit("eval", i)
        cands = sv.sv_tune_candidates(n, dtype)
        ncand = len(cands)
        cold_compile_s = float(sum(csec[k:k + ncand]))
        k += ncand + 1
        st = sv.StateVector(n, dtype)
        t1 = time.perf_counter()
        pick = sv.sv_tune(st.h, g, sv.SV_TUNER_LEARNED)
        learned_tune_s = time.perf_counter() - t1
        li = [_fields(c) for c in cands].index(_fields(pick))
        try:
            # one candidate per call, each logged: a large state times for minutes
            ms = []
            for j, c in enumerate(cands):
                ms += sv.sv_tune_time(st.h, g, [c], repeats)[0]
                log(f"eval {i} n={n}: candidate {j + 1}/{ncand} {ms[-1]:.1f} ms")
            pms, _ = sv.sv_tune_time(st.h, g, [sv.paper_schedule(paper_l)], repeats)
        except sv.SvError as e:
            st.close()
            if e.status != sv.SV_ERR_OUT_OF_MEMORY:
                raise
            log(f"eval {i} n={n}: not measured ({e.message})")
            per.append({"circuit": i, "n": n, "learned": li, "not_measured": e.message})
            release()
            continue
        st.close()
        release()
        best = int(np.argmin(ms))
        rec = {"circuit": i, "n": n, "ms": ms, "best": best, "learned": li,
               "regret": ms[li] / ms[best] - 1.0, "paper_ms": pms[0],
               "gain_vs_paper": pms[0] / ms[li],
               "exhaustive_tune_s": cold_compile_s + sum(ms) * (repeats + 1) / 1e3,
               "learned_tune_s": learned_tune_s + cold_compile_s / ncand}
        per.append(rec)
        log(f"eval {i} n={n}: best {ms[best]:.1f} ms, learned {ms[li]:.1f} ms "
            f"(regret {100 * rec['regret']:.1f}%), paper {pms[0]:.1f} ms")
    done = [r for r in per if "regret" in r]
    reg = np.array([r["regret"] for r in done])
    return {"model": meta, "circuits": per, "measured": len(done),
            "regret_median": float(np.median(reg)), "regret_p90": float(np.percentile(reg, 90)),
            "picked_best": int(sum(r["learned"] == r["best"] for r in done)),
            "gain_vs_paper_median": float(np.median([r["gain_vs_paper"] for r in done])),
            "exhaustive_tune_s_median": float(np.median([r["exhaustive_tune_s"] for r in done])),
            "learned_tune_s_median": float(np.median([r["learned_tune_s"] for r in done]))}


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
    c.add_argument("--workers", type=int, default=12)
    c.add_argument("--out", required=True)
    t = sub.add_parser("train")
    t.add_argument("--data", required=True, help="one or more collected .npz files, comma separated")
    t.add_argument("--epochs", type=int, default=400)
    t.add_argument("--out", required=True)
    e = sub.add_parser("eval")
    e.add_argument("--model", default=MODEL_PATH)
    e.add_argument("--per-n", type=int, default=5)
    e.add_argument("--circuits", default="", help="explicit eval circuits a:b (instead of --per-n)")
    e.add_argument("--workers", type=int, default=12)
    e.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "collect":
        lo, hi = a.qubits.split(":")
        kind = "train" if (lo, hi) == ("20", "26") else f"train:{lo}:{hi}"
        d = collect(_range(a.circuits), workers=a.workers, kind=kind)
        np.savez(a.out, **d)
        log(f"wrote {a.out}")
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
                "final_train_mse": hist[-1],
                "train_mse_check": float(np.mean((pred - np.log(ms)) ** 2))}
        save(a.out, params, norm, meta)
        log(f"wrote {a.out}: {meta}")
    else:
        idxs = _range(a.circuits) if a.circuits else [10 * k + j for k in range(5) for j in range(a.per_n)]
        res = evaluate(idxs, a.model, workers=a.workers)
        with open(a.out, "w") as fh:
            json.dump(res, fh, indent=1)
        log(f"regret median {res['regret_median']:.3f}, p90 {res['regret_p90']:.3f}, "
            f"picked best {res['picked_best']}/{res['measured']}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
