"""Benchmark: solves/s of the coordinate-descent L-MMSE detector (Algorithm 1) on one
MI355X, to a fixed relative tolerance against the FP64 CPU oracle.

Workload (default): one dense uplink instance, B = 16384 antennas x U = 8192 users,
complex128, H ~ CN(0, 1/16384), y ~ CN(0, 1), seed 1, lambda = N0/Ex = 0.1;
iterate until the relative step sqrt(sum |delta_u|^2)/||x|| <= 1e-11 (cap 200
sweeps), which puts the result within 1e-10 of the FP64 oracle's.  The mixed
precisions (--precision bf16 | fp8) cap the refinement at ceil(200 / k) outer steps of
k low-precision sweeps each (k = 12 for BF16, 5 for FP8): the same 200-sweep cap,
counted in sweeps over the copy.  One step = one
complete solve through the C ABI: column energies and panel Gram inverses, init,
all sweeps, finalisation.  Inputs are resident in HBM before timing starts.

Prints ONE JSON line.  `value` = solves/s; `roofline` is for the sweep kernel
(algorithmic bytes = one read of H per sweep) timed with HIP events on the solve's
stream; `cpu_baseline` is the FP64 oracle timed on this host (one thread).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch (per solve) from rocprofv3 FETCH_SIZE and WRITE_SIZE passes scaled by
# the copy-kernel calibration (profiles/), valid only while the sources that make the
# kernel hash to the recorded value.
TRAFFIC = {
    ("k_cd_panel_la", "c128 16384x8192 tol 1e-11"): {
        "sources": ['paper_1902_08653_amd/csrc/k_panel_la.hip', 'paper_1902_08653_amd/csrc/la_common.hpp', 'paper_1902_08653_amd/csrc/panel.hpp', 'paper_1902_08653_amd/csrc/common.hpp'], "sha256_16": "7c6f7e01785c5fb6", "bytes": 143080384512.0},
    ("k_cd_wg", "c64 batch 4096 tol 1e-06"): {
        "sources": ['paper_1902_08653_amd/csrc/k_wg.hip', 'paper_1902_08653_amd/csrc/common.hpp', 'paper_1902_08653_amd/csrc/wg.hpp'], "sha256_16": "247b0c159f0cd8bb", "bytes": 713278845676.0},
    ("k_cd_sparse", "c128 16384x8192 0.01 tol 1e-11"): {
        "sources": ['paper_1902_08653_amd/csrc/k_sparse.hip', 'paper_1902_08653_amd/csrc/common.hpp', 'paper_1902_08653_amd/csrc/launch.hpp'], "sha256_16": "3b4e73b3b5f40875", "bytes": 9869837984.0},
    ("k_bm_resid + k_bm_grad + k_bm_inner", "mixed-c64 batch 4096 tol 1e-08"): {
        "sources": ['paper_1902_08653_amd/csrc/k_wg_mixed.hip', 'paper_1902_08653_amd/csrc/common.hpp', 'paper_1902_08653_amd/csrc/wg.hpp', 'paper_1902_08653_amd/csrc/quant.hpp'], "sha256_16": "a27fee61a3afae15", "bytes": 1178767779708.0},
}


def measured_traffic(kernel, workload):
    import hashlib
    rec = TRAFFIC.get((kernel, workload))
    if rec is None:
        return None
    sha = hashlib.sha256()
    for f in rec["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            sha.update(fh.read())
    return rec["bytes"] if sha.hexdigest()[:16] == rec["sha256_16"] else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--B", type=int, default=16384)
    ap.add_argument("--U", type=int, default=8192)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--precision", default=None, choices=["c128", "c64", "bf16", "fp8", "mixed-c64"],
                    help="dense (default c128): c128/c64 plain sweeps, bf16/fp8 mixed-precision refinement "
                         "(FP64 outer gradient around FP32 inner sweeps on a BF16/FP8 copy); batched (default "
                         "c64): c64/c128 plain, mixed-c64/bf16 mixed-precision refinement")
    ap.add_argument("--tol", type=float, default=None)
    ap.add_argument("--eps", type=float, default=None, help="accuracy target vs the oracle")
    ap.add_argument("--lam", type=float, default=0.1)
    ap.add_argument("--lookahead", default="one", choices=["one", "deep", "none"],
                    help="dense panel engine schedule: one panel ahead, two panels ahead, or two-hop")
    ap.add_argument("--no-oracle", action="store_true", help="skip the oracle check and CPU baseline")
    ap.add_argument("--cpu-sweeps", type=int, default=0,
                    help="oracle sweeps for the CPU baseline (0 = a full solve)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="accepted for old command lines: the read and copy probes always run")
    ap.add_argument("--workload", default="dense", choices=["dense", "batched", "warm", "paper", "sparse"],
                    help="dense: one 16384x8192 instance (default); batched: 4096 uneven instances; "
                         "warm: learned warm start against a cold start on 4096 held-out uneven instances; "
                         "paper: the paper's uplink throughput shape; sparse: one 16384x8192 CSR instance")
    ap.add_argument("--density", type=float, default=0.01, help="sparse: nonzero density")
    ap.add_argument("--train", type=int, default=50000, help="warm: training instances")
    ap.add_argument("--epochs", type=int, default=3, help="warm: training epochs")
    ap.add_argument("--inner", default="c64", choices=["c64", "bf16"],
                    help="warm: inner copy of the mixed-precision form")
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--sample", type=int, default=0,
                    help="batched: instances checked against the oracle (0 = all of them)")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: multi-GPU runs are not part of this build "
              "(the instances shard by cluster or by instance with no exchange during the sweeps)",
              file=sys.stderr)
        sys.exit(2)
    if a.workload == "batched":
        return bench_batched(a)
    if a.workload == "warm":
        return bench_warm(a)
    if a.workload == "paper":
        return bench_paper(a)
    if a.workload == "sparse":
        return bench_sparse(a)
    import torch

    from paper_1902_08653_amd import cdm, inputs

    prec = a.precision or "c128"
    if prec == "mixed-c64":
        sys.exit("dense workload: --precision c128, c64, bf16 or fp8")
    fp64_target = prec in ("c128", "bf16", "fp8")
    tol = a.tol if a.tol is not None else (1e-11 if fp64_target else 1e-6)
    eps = a.eps if a.eps is not None else (1e-10 if fp64_target else 1e-5)
    dev = torch.device("cuda:0")
    t0 = time.time()
    inst = inputs.dense_uplink(a.B, a.U, a.seed)
    npdt = np.complex128 if fp64_target else np.complex64
    Hc = torch.from_numpy(np.ascontiguousarray(inst.H.T).astype(npdt, copy=False)).to(dev)
    y = torch.from_numpy(inst.y.astype(npdt)).to(dev)
    print("[bench] inputs ready in %.1fs" % (time.time() - t0), file=sys.stderr, flush=True)

    # the mixed precisions' T_max counts outer refinement steps of k inner sweeps each:
    # the same cap of 200 sweeps, counted over the low-precision copy
    inner = cdm.MIXED_INNER_SWEEPS.get(prec, 0)
    cap = -(-200 // inner) if inner else 200
    plan = cdm.Plan(a.B, a.U, precision=prec, T_max=cap, tol=tol, timing=True,
                    lookahead={"one": True, "deep": "deep", "none": False}[a.lookahead])
    stream = torch.cuda.current_stream()
    x = torch.empty(a.U, dtype=y.dtype, device=dev)
    info = torch.empty(32, dtype=torch.uint8, device=dev)
    for _ in range(a.warmup):
        plan.solve(Hc, y, N0=a.lam, Ex=1.0, x=x, info=info)
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    stage = {k: 0.0 for k in cdm.Plan.STAGES}
    sweeps = []
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    wall0 = time.perf_counter()
    for _ in range(a.steps):
        plan.solve(Hc, y, N0=a.lam, Ex=1.0, x=x, info=info)
        # per-stage events of this solve; reading them needs the stream drained
        torch.cuda.synchronize()
        for k, v in plan.timings().items():
            stage[k] += v
        sweeps.append(int(cdm.parse_info(info)[0]["sweeps"]))
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = ev0.elapsed_time(ev1)
    ms_per = ms_total / a.steps
    rec = cdm.parse_info(info)[0]
    xg = x.cpu().numpy().astype(np.complex128)
    resid = plan.residual(Hc, y, x, N0=a.lam).item()
    torch.cuda.synchronize()
    print("[bench] timed %d solves: %.3f ms/solve, sweeps %s" % (a.steps, ms_per, sweeps),
          file=sys.stderr, flush=True)

    esz = 16 if prec == "c128" else 8
    h_bytes = float(a.B) * a.U * esz
    if prec in ("bf16", "fp8"):
        # one outer step reads the complex128 H twice (residual, gradient) and runs the
        # inner sweeps over the 4-byte (BF16) or 2-byte (FP8) planar copy
        qb = 4.0 if prec == "bf16" else 2.0
        h_bytes = float(a.B) * a.U * (2 * 16 + inner * qb)
    desc = json.loads(plan.describe())
    sweep_kernel = "k_cd_panel_la" if desc.get("schedule") == "lookahead" else (
        "k_cd_panel" if desc.get("engine") == "panel" else "k_cd_wg")
    if desc.get("lookahead_panels") == 2:
        sweep_kernel = "k_cd_panel_deep"
    if prec in ("bf16", "fp8"):
        sweep_kernel = "outer refinement loop (k_mx_* FP64 passes + k_cd_panel_la inner sweeps)"
    sweep_ms = stage["sweeps"] / a.steps
    mean_sweeps = float(np.mean(sweeps))
    achieved = mean_sweeps * h_bytes / (sweep_ms * 1e-3) / 1e9

    probes = _hbm_probes(cdm, dev, stream)

    oracle_err = None
    cpu = None
    if not a.no_oracle:
        from oracle import oracle
        H64 = inst.H.astype(npdt).astype(np.complex128) if prec != "c128" else inst.H
        y64 = inst.y.astype(npdt).astype(np.complex128) if prec != "c128" else inst.y
        oracle.build()
        tc = time.perf_counter()
        if a.cpu_sweeps > 0:
            ref = oracle.local_cd(H64, y64, a.lam, T_max=a.cpu_sweeps)
        else:
            ref = oracle.local_cd(H64, y64, a.lam, T_max=200, tol=tol)
        cpu_s = time.perf_counter() - tc
        print("[bench] oracle %d sweeps in %.1fs" % (ref["sweeps"], cpu_s), file=sys.stderr, flush=True)
        # plain sweeps: the oracle's time per sweep times this solve's sweep count; mixed
        # precision: the oracle's own solve to the same tolerance
        per_solve = cpu_s / ref["sweeps"] * (mean_sweeps if prec in ("c128", "c64") else ref["sweeps"])
        scaled = mean_sweeps if prec in ("c128", "c64") else float(ref["sweeps"])
        cpu = {"value": 1.0 / per_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": "%d oracle sweeps of the same %dx%d instance (%.1f s, single thread), "
                         "scaled to %.1f sweeps per solve" % (ref["sweeps"], a.B, a.U, cpu_s, scaled)}
        if a.cpu_sweeps == 0:
            oracle_err = float(np.linalg.norm(xg - ref["x"]) / np.linalg.norm(ref["x"]))

    out = {
        "metric": "solves/sec to fixed rel. tolerance vs FP64 oracle",
        "value": 1000.0 / ms_per,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"c128": "f64", "c64": "f32", "bf16": "bf16+f32+f64", "fp8": "fp8+f32+f64"}[prec],
        "data": "synthetic",
        "config": {"workload": "dense uplink L-MMSE CD (Algorithm 1), B=%d antennas x U=%d users, "
                               "%s, CN(0,1/B) channel, seed %d, lambda=%g, rel-step tol %g, %s"
                               % (a.B, a.U, prec, a.seed, a.lam, tol,
                                  "cap %d outer steps x %d inner sweeps" % (cap, inner) if inner else "cap 200"),
                   "B": a.B, "U": a.U, "precision": prec, "tol": tol, "eps": eps,
                   "engine": json.loads(plan.describe())},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(sweep_kernel, "%s %dx%d tol %g" % (prec, a.B, a.U, tol)),
                     "kernel": sweep_kernel, "algorithmic_bytes_per_launch": mean_sweeps * h_bytes,
                     "avg_launch_ms": sweep_ms, **_ceiling(achieved, probes)},
        "cpu_baseline": cpu,
        "accuracy": {"sweeps": sweeps, "rel_step": float(rec["rel_step"]), "flags": int(rec["flags"]),
                     "fp64_normal_residual": resid, "rel_err_vs_oracle": oracle_err,
                     "within_eps": (oracle_err is not None and oracle_err <= eps)},
        "stages_ms_per_solve": {k: v / a.steps for k, v in stage.items()},
        "wall_s_timed": wall,
    }
    out["copy_probe_gbs"] = probes["copy_gbs"]
    out.setdefault("host", _host_info())
    print(json.dumps(out))
    plan.close()


def bench_batched(a):
    """4096 independent uplink instances, m ~ U{64..2048}, n = m/2, lambda 0.1, in one
    HIP graph.  --precision c64 (the default here): complex64 data, plain sweeps to a
    relative step of 1e-6 in one persistent launch.  c128: complex128 data, plain sweeps
    to 1e-8.  mixed-c64 / bf16: complex128 data, the mixed-precision refinement (complex64
    or BF16 inner copy) to 1e-8.  Tiles from the library's autotuner."""
    import torch

    from paper_1902_08653_amd import cdm, inputs
    dev = torch.device("cuda:0")
    prec = a.precision or "c64"
    if prec not in ("c64", "c128", "mixed-c64", "bf16"):
        sys.exit("batched workload: --precision c64, c128, mixed-c64 or bf16")
    c64 = prec == "c64"
    mixed = prec in ("mixed-c64", "bf16")
    tol, eps = (1e-6, 1e-5) if c64 else (1e-8, 1e-6)
    dt = torch.complex64 if c64 else torch.complex128
    esz = 8 if c64 else 16
    t0 = time.time()
    H, y, m, n = inputs.batch_uneven_device(a.batch, seed0=0, dtype=dt, device=dev)
    torch.cuda.synchronize()
    print("[bench] batch of %d ready in %.1fs (%.2f GB)" % (a.batch, time.time() - t0, H.numel() * esz / 1e9),
          file=sys.stderr, flush=True)
    plan = cdm.BatchedPlan(m, n, precision=prec, T_max=(8 if prec == "mixed-c64" else 16) if mixed else 200,
                           tol=tol, autotune=True)
    x = torch.empty(int(n.astype(np.int64).sum()), dtype=dt, device=dev)
    info = torch.empty(32 * a.batch, dtype=torch.uint8, device=dev)
    g = _graph(lambda: plan.solve(H, y, N0=a.lam, x=x, info=info))
    ms = _time_graph(g, a.steps, a.warmup)
    rec = cdm.parse_info(info)
    sweeps = rec["sweeps"].astype(np.int64)
    mn = m.astype(np.int64) * n.astype(np.int64)
    if mixed:
        lowsz = 8 if prec == "mixed-c64" else 4
        inner = rec["reserved"].astype(np.int64)
        # FP64 passes (a cold first step needs only g), inner sweeps over the copy, its write
        alg_bytes = float((mn * (16 * (2 * sweeps - 1) + lowsz * inner + lowsz)).sum())
        kernel = "k_bm_resid + k_bm_grad + k_bm_inner"
        acc = {"outer_mean": float(sweeps.mean()), "inner_sweeps_mean": float(inner.mean())}
    else:
        alg_bytes = float((sweeps * mn * esz).sum())
        kernel = "k_cd_wg"
        acc = {"sweeps_mean": float(sweeps.mean()), "sweeps_max": int(sweeps.max())}
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    probes = _hbm_probes(cdm, dev, torch.cuda.current_stream())
    print("[bench] %.3f ms per batch solve, %s, flags %d" % (ms, acc, int(np.bitwise_or.reduce(rec["flags"]))),
          file=sys.stderr, flush=True)
    cpu = None
    errs = []
    if not a.no_oracle:
        errs, cpu = _batched_oracle_check(a, H, y, x, m, n, sweeps, mixed, c64, tol)
    out = {
        "metric": "solves/sec to fixed rel. tolerance vs FP64 oracle",
        "value": a.batch * 1000.0 / ms,
        "unit": "instance solves/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"c64": "f32", "c128": "f64", "mixed-c64": "f32+f64", "bf16": "bf16+f32+f64"}[prec],
        "data": "synthetic",
        "config": {"workload": "%d uneven uplink instances, m~U{64..2048}, n=m/2, %s, CN(0,1/m), lambda=%g, "
                               "rel-step tol %g, HIP graph" % (a.batch, prec, a.lam, tol),
                   "engine": json.loads(plan.describe())},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(kernel, "%s batch %d tol %g" % (prec, a.batch, tol)),
                     "kernel": kernel, "algorithmic_bytes_per_launch": alg_bytes, "avg_launch_ms": ms,
                     **_ceiling(achieved, probes)},
        "cpu_baseline": cpu,
        "accuracy": dict(acc, flags_or=int(np.bitwise_or.reduce(rec["flags"])),
                         instances_checked=len(errs),
                         max_rel_err_vs_oracle=max(errs) if errs else None,
                         instances_within_eps=int(np.sum(np.asarray(errs) <= eps)) if errs else None,
                         within_eps=bool(max(errs) <= eps) if errs else None),
        "host": _host_info(),
    }
    out["copy_probe_gbs"] = probes["copy_gbs"]
    out.setdefault("host", _host_info())
    print(json.dumps(out))
    plan.close()


def _host_info():
    """Host cores and CPU model, printed beside every CPU figure."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"nproc": avail, "cpu_count": os.cpu_count(), "cpu_model": model}


def _oracle_threads():
    # the machine's CPU share is 16 cores per GPU, whatever the OS reports
    return max(1, min(16, _host_info()["nproc"] or 1))


def _batched_oracle_check(a, H, y, x, m, n, sweeps, mixed, c64, tol):
    """Every instance of the batch (or --sample of them, spread over the sizes) against
    the FP64 oracle, on a pool of host threads (the oracle is C behind ctypes, which
    drops the GIL for the call).  The same pool's wall time for the oracle's own solves
    at the bench's stop rule is the CPU baseline."""
    import concurrent.futures as cf

    from oracle import oracle
    oracle.build()
    mn = m.astype(np.int64) * n.astype(np.int64)
    ho = np.concatenate([[0], np.cumsum(mn)[:-1]])
    yo = np.concatenate([[0], np.cumsum(m.astype(np.int64))[:-1]])
    xo = np.concatenate([[0], np.cumsum(n.astype(np.int64))[:-1]])
    if a.sample and a.sample < a.batch:
        order = np.argsort(-mn)
        pick = order[np.linspace(0, a.batch - 1, a.sample).astype(int)]
    else:
        pick = np.arange(a.batch)
    xg = x.cpu().numpy()
    nthr = _oracle_threads()

    def chunks():
        """Device -> host in runs of consecutive instances (one copy per run), so the
        copies keep ahead of the oracle threads."""
        k = 0
        while k < len(pick):
            j = k + 1
            while j < len(pick) and j - k < 64 and pick[j] == pick[j - 1] + 1:
                j += 1
            i0, i1 = int(pick[k]), int(pick[j - 1])
            Hh = H[ho[i0]:ho[i1] + mn[i1]].cpu().numpy()
            yh = y[yo[i0]:yo[i1] + m[i1]].cpu().numpy()
            for i in range(i0, i1 + 1):
                yield (i, Hh[ho[i] - ho[i0]:ho[i] - ho[i0] + mn[i]], yh[yo[i] - yo[i0]:yo[i] - yo[i0] + m[i]])
            k = j

    def pool_pass(job):
        out = []
        t = time.perf_counter()
        with cf.ThreadPoolExecutor(nthr) as pool:
            pending = set()
            for i, Hf, yf in chunks():
                pending.add(pool.submit(job, i, Hf, yf))
                if len(pending) >= 8 * nthr:
                    done, pending = cf.wait(pending, return_when=cf.FIRST_COMPLETED)
                    out.extend(f.result() for f in done)
            out.extend(f.result() for f in cf.as_completed(pending))
        return out, time.perf_counter() - t

    def inputs_of(i, Hf, yf):
        # column-major m x n from the packed slice, promoted to complex128 for the oracle
        return Hf.reshape(n[i], m[i]).T.astype(np.complex128), yf.astype(np.complex128)

    def err(i, ref):
        got = xg[xo[i]:xo[i] + n[i]]
        return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))

    def at_tol(i, Hf, yf):
        Hi, yi = inputs_of(i, Hf, yf)
        ref = oracle.local_cd(Hi, yi, a.lam, T_max=200, tol=tol)
        return (err(i, ref["x"]) if c64 else None), int(ref["sweeps"])

    def exact(i, Hf, yf):
        Hi, yi = inputs_of(i, Hf, yf)
        return err(i, oracle.local_cd(Hi, yi, a.lam, T_max=2000, tol=1e-13)["x"]), 0

    res, cpu_s = pool_pass(at_tol)
    osweeps = sum(r[1] for r in res)
    if c64:
        errs = [r[0] for r in res]
    else:
        # complex128 forms are held to the converged solution (a second, untimed pass)
        errs = [r[0] for r in pool_pass(exact)[0]]
    print("[bench] oracle checked %d instances on %d threads (%.1fs at the stop rule): max rel err %.3e"
          % (len(pick), nthr, cpu_s, max(errs)), file=sys.stderr, flush=True)
    cpu = {"value": len(pick) / cpu_s, "unit": "instance solves/s", "cores": nthr, "kind": "oracle",
           "sample": "%d of %d instances, FP64 oracle to rel. step %g (%d oracle sweeps in all) on a pool of "
                     "%d host threads, %.1f s wall" % (len(pick), a.batch, tol, osweeps, nthr, cpu_s)}
    return errs, cpu


def bench_sparse(a):
    """One sparse uplink instance, B x U (default 16384 x 8192) at density 1 %
    (Bernoulli pattern, nonzeros CN(0, 1/(0.01 B)), int32 CSR, seed 1), lambda 0.1,
    complex128 (or complex64), plain sweeps to a relative step of 1e-11 (1e-6 for
    complex64), cap 200.  One step = one solve through the C ABI from the CSR arrays:
    transpose to columns, sparse panel Gram and inverses, init, all sweeps, finalise."""
    import torch

    from paper_1902_08653_amd import cdm, inputs
    dev = torch.device("cuda:0")
    prec = a.precision or "c128"
    if prec not in ("c128", "c64"):
        sys.exit("sparse workload: --precision c128 or c64")
    density = a.density
    tol = a.tol if a.tol is not None else (1e-11 if prec == "c128" else 1e-6)
    eps = a.eps if a.eps is not None else (1e-10 if prec == "c128" else 1e-5)
    npdt = np.complex128 if prec == "c128" else np.complex64
    esz = 16 if prec == "c128" else 8
    t0 = time.time()
    ins = inputs.sparse_uplink(a.B, a.U, density, seed=a.seed, dtype=npdt)
    nnz = int(ins.rowptr[-1])
    val = torch.from_numpy(ins.val.astype(npdt)).to(dev)
    rp = torch.from_numpy(ins.rowptr).to(dev)
    ci = torch.from_numpy(ins.colidx).to(dev)
    y = torch.from_numpy(ins.y.astype(npdt)).to(dev)
    print("[bench] sparse %dx%d, nnz %d, ready in %.1fs" % (a.B, a.U, nnz, time.time() - t0),
          file=sys.stderr, flush=True)
    plan = cdm.Plan(a.B, a.U, layout="csr", nnz=nnz, precision=prec, T_max=200, tol=tol, timing=True)
    stream = torch.cuda.current_stream()
    x = torch.empty(a.U, dtype=y.dtype, device=dev)
    info = torch.empty(32, dtype=torch.uint8, device=dev)
    for _ in range(a.warmup):
        plan.solve(val, y, N0=a.lam, x=x, info=info, rowptr=rp, colidx=ci)
    torch.cuda.synchronize()
    stage = {k: 0.0 for k in cdm.Plan.STAGES}
    sweeps = []
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(a.steps):
        plan.solve(val, y, N0=a.lam, x=x, info=info, rowptr=rp, colidx=ci)
        torch.cuda.synchronize()
        for k, v in plan.timings().items():
            stage[k] += v
        sweeps.append(int(cdm.parse_info(info)[0]["sweeps"]))
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_per = ev0.elapsed_time(ev1) / a.steps
    rec = cdm.parse_info(info)[0]
    xg = x.cpu().numpy().astype(np.complex128)
    sweep_ms = stage["sweeps"] / a.steps
    mean_sweeps = float(np.mean(sweeps))
    # per sweep: the column values and row indices are read once to gather r and once to
    # scatter the panel's update back into r
    alg_bytes = mean_sweeps * 2.0 * nnz * (esz + 4)
    achieved = alg_bytes / (sweep_ms * 1e-3) / 1e9
    probes = _hbm_probes(cdm, dev, stream)
    print("[bench] %.3f ms per solve (sweep kernel %.3f ms), sweeps %s" % (ms_per, sweep_ms, sweeps),
          file=sys.stderr, flush=True)
    cpu = None
    err = None
    if not a.no_oracle:
        from oracle import oracle
        oracle.build()
        v64 = ins.val.astype(np.complex128)
        y64 = ins.y.astype(npdt).astype(np.complex128)
        # whole oracle solves of the same instance, repeated for about 10 s
        reps = 0
        tc = time.perf_counter()
        while True:
            colptr, rowidx, cval = oracle.csr_to_csc(a.B, a.U, ins.rowptr, ins.colidx, v64)
            ref = oracle.local_cd_csc(a.B, a.U, colptr, rowidx, cval, y64, a.lam, T_max=200, tol=tol)
            reps += 1
            cpu_s = time.perf_counter() - tc
            if cpu_s >= 10.0 or reps >= 200:
                break
        err = float(np.linalg.norm(xg - ref["x"]) / np.linalg.norm(ref["x"]))
        cpu = {"value": reps / cpu_s, "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": "%d full oracle solves of the same instance (CSR to columns and %d sweeps to "
                         "rel. step %g each; %.1f s, single thread)" % (reps, ref["sweeps"], tol, cpu_s)}
        print("[bench] oracle %d sweeps in %.2fs, rel err %.2e" % (ref["sweeps"], cpu_s, err),
              file=sys.stderr, flush=True)
    out = {
        "metric": "solves/sec to fixed rel. tolerance vs FP64 oracle",
        "value": 1000.0 / ms_per,
        "unit": "solves/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_per,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == "c128" else "f32",
        "data": "synthetic",
        "config": {"workload": "sparse uplink L-MMSE CD (Algorithm 1), B=%d x U=%d, density %g, int32 CSR, "
                               "%s, CN(0,1/(%g B)) nonzeros, seed %d, lambda=%g, rel-step tol %g, cap 200"
                               % (a.B, a.U, density, prec, density, a.seed, a.lam, tol),
                   "B": a.B, "U": a.U, "nnz": nnz, "precision": prec, "tol": tol, "eps": eps,
                   "engine": json.loads(plan.describe())},
        # frac against HBM is reported as measured; the sweep is a
        # chain of panel steps (partial, exchange across the slice workgroups, panel product,
        # scatter) over a MALL-resident operator, so its limiter is that chain's latency
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("k_cd_sparse", "%s %dx%d %g tol %g" % (prec, a.B, a.U, density, tol)),
                     "kernel": "k_cd_sparse",
                     "limiter": "per-panel exchange latency across the slice workgroups, not HBM",
                     "algorithmic_bytes_per_launch": alg_bytes, "avg_launch_ms": sweep_ms,
                     **_ceiling(achieved, probes)},
        "cpu_baseline": cpu,
        "accuracy": {"sweeps": sweeps, "rel_step": float(rec["rel_step"]), "flags": int(rec["flags"]),
                     "rel_err_vs_oracle": err, "within_eps": (err is not None and err <= eps)},
        "stages_ms_per_solve": {k: v / a.steps for k, v in stage.items()},
    }
    out["copy_probe_gbs"] = probes["copy_gbs"]
    out.setdefault("host", _host_info())
    print(json.dumps(out))
    plan.close()


# the paper's Table I (uplink detector, latency ms / throughput Gbit/s on C V100 GPUs
# including the inter-GPU fusion): context for the paper-shaped workload, not a target
PAPER_TABLE_I = {("fp32", 4, 2): (0.465, 1.23), ("fp32", 4, 3): (0.540, 1.06), ("fp32", 4, 4): (0.617, 0.93),
                 ("fp32", 8, 2): (0.502, 1.14), ("fp32", 8, 3): (0.585, 0.98), ("fp32", 8, 4): (0.665, 0.86),
                 ("fp16", 4, 2): (0.259, 2.21), ("fp16", 4, 3): (0.298, 1.92), ("fp16", 4, 4): (0.341, 1.68),
                 ("fp16", 8, 2): (0.295, 1.95), ("fp16", 8, 3): (0.331, 1.73), ("fp16", 8, 4): (0.370, 1.55)}


# the downlink half of Table I (precoding, same shapes; latency ms / throughput Gbit/s)
PAPER_TABLE_I_DL = {("fp32", 4, 2): (0.414, 1.38), ("fp32", 4, 3): (0.499, 1.15), ("fp32", 4, 4): (0.577, 0.99),
                    ("fp32", 8, 2): (0.440, 1.30), ("fp32", 8, 3): (0.525, 1.09), ("fp32", 8, 4): (0.601, 0.95),
                    ("fp16", 4, 2): (0.228, 2.52), ("fp16", 4, 3): (0.267, 2.15), ("fp16", 4, 4): (0.305, 1.88),
                    ("fp16", 8, 2): (0.233, 2.46), ("fp16", 8, 3): (0.275, 2.09), ("fp16", 8, 4): (0.311, 1.84)}


def bench_paper(a):
    """The paper's throughput shape on one GPU: 1200 subcarriers x 15 received vectors,
    U = 8 users, 16-QAM, Rayleigh channels, C clusters of 32 antennas, T sweeps from
    x = 0, cluster fusion; one cdm_detect_batch launch per batch (HIP graph replays).
    The headline line is C = 4, T = 3 in FP16 (the configuration of the paper's
    per-user throughput comparison); every (C, T, precision) cell is reported, and the
    downlink half of the table (cdm_precode_batch on the same shape) beside it."""
    import torch

    from paper_1902_08653_amd import cdm, inputs
    dev = torch.device("cuda:0")
    S, V, U, Bc = 1200, 15, 8, 32
    bits = S * V * U * 4
    cells, lines, dl = {}, [], {}
    for Cn in (4, 8):
        d = inputs.paper_shaped(Cn, Bc, U, S, V, snr_db=10.0, seed=1)
        B = Cn * Bc
        H32 = torch.from_numpy(d["Ht"].astype(np.complex64).reshape(-1)).to(dev)
        Y32 = torch.from_numpy(d["Y"].astype(np.complex64).reshape(-1)).to(dev)
        H16 = torch.from_numpy(np.stack([d["Ht"].real, d["Ht"].imag], -1).astype(np.float16).reshape(-1)).to(dev)
        Y16 = torch.from_numpy(np.stack([d["Y"].real, d["Y"].imag], -1).astype(np.float16).reshape(-1)).to(dev)
        X32 = torch.from_numpy(d["X"].astype(np.complex64).reshape(-1)).to(dev)
        X16 = torch.from_numpy(np.stack([d["X"].real, d["X"].imag], -1).astype(np.float16).reshape(-1)).to(dev)
        for prec, (Hd, Yd, Xd, esz) in (("fp32", (H32, Y32, X32, 8)), ("fp16", (H16, Y16, X16, 4))):
            out = torch.empty(S * V * U * (1 if prec == "fp32" else 2), dtype=Yd.dtype, device=dev)
            pre = torch.empty(S * V * B * (1 if prec == "fp32" else 2), dtype=Yd.dtype, device=dev)
            for T in (2, 3, 4):
                g = _graph(lambda: cdm.precode_batch(Hd, Xd, S, V, Cn, Bc, U, T, 1.0, out=pre))
                ms = _time_graph(g, max(a.steps, 50), max(a.warmup, 5))
                del g
                algo = (S * B * U + S * V * U + S * V * B) * esz
                dl[(prec, Cn, T)] = dict(ms=ms, gbps=bits / (ms * 1e-3) / 1e9, hbm_gbs=algo / (ms * 1e-3) / 1e9,
                                         bytes=algo)
                pl, pt = PAPER_TABLE_I_DL[(prec, Cn, T)]
                print("[bench] downlink %s C=%d T=%d: %.4f ms, %.1f Gbit/s (paper on %d V100: %.3f ms, %.2f Gbit/s)"
                      % (prec, Cn, T, ms, dl[(prec, Cn, T)]["gbps"], Cn, pl, pt), file=sys.stderr, flush=True)
                g = _graph(lambda: cdm.detect_batch(Hd, Yd, S, V, Cn, Bc, U, T, d["N0"], out=out))
                ms = _time_graph(g, max(a.steps, 50), max(a.warmup, 5))
                del g
                algo = (S * B * U + S * V * B + S * V * U) * esz
                cells[(prec, Cn, T)] = dict(ms=ms, gbps=bits / (ms * 1e-3) / 1e9, hbm_gbs=algo / (ms * 1e-3) / 1e9,
                                            bytes=algo)
                pl, pt = PAPER_TABLE_I[(prec, Cn, T)]
                lines.append("%s C=%d T=%d: %.4f ms, %.1f Gbit/s (paper on %d V100: %.3f ms, %.2f Gbit/s)"
                             % (prec, Cn, T, ms, cells[(prec, Cn, T)]["gbps"], Cn, pl, pt))
                print("[bench] " + lines[-1], file=sys.stderr, flush=True)
    head = cells[("fp16", 4, 3)]
    cpu = None
    if not a.no_oracle:
        from oracle import oracle
        oracle.build()
        d = inputs.paper_shaped(4, Bc, U, 40, V, snr_db=10.0, seed=1)
        tc = time.perf_counter()
        n = 0
        for s_ in range(40):
            H = d["Ht"][s_].T.astype(np.complex128)
            for v in range(V):
                oracle.uplink_cd(H, d["Y"][s_, v].astype(np.complex128), d["N0"], 1.0, T_max=3, C_clusters=4)
                n += 1
        cs = time.perf_counter() - tc
        cpu = {"value": n * U * 4 / cs / 1e9, "unit": "Gbit/s", "cores": 1, "kind": "oracle",
               "sample": "%d of the batch's received vectors (C = 4, T = 3) through the oracle's Algorithm 1 "
                         "with fusion on one thread (%.2f s)" % (n, cs)}
    out = {
        "metric": "detection throughput of the paper's Table I batch",
        "value": head["gbps"], "unit": "Gbit/s",
        "n_gpus": 1, "steps": max(a.steps, 50), "warmup": max(a.warmup, 5), "ms_per_step": head["ms"],
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": head["gbps"] / PAPER_TABLE_I[("fp16", 4, 3)][1],
        "vs_baseline_note": "paper's Table I on 4 V100 GPUs incl. inter-GPU fusion; context, not the target",
        "dtype": "f16", "data": "synthetic",
        "config": {"workload": "paper-shaped uplink: 1200 subcarriers x 15 vectors, U=8, 16-QAM, Rayleigh, "
                               "C=4 clusters x 32 antennas, T=3, fusion, SNR 10 dB"},
        "roofline": {"bound": "hbm", "achieved": head["hbm_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": head["hbm_gbs"] / HBM_PEAK_GBS, "traffic": None, "kernel": "k_detect_small",
                     "algorithmic_bytes_per_launch": head["bytes"], "avg_launch_ms": head["ms"]},
        "cpu_baseline": cpu,
        "cells": {"%s_C%d_T%d" % k: v for k, v in cells.items()},
        "downlink_cells": {"%s_C%d_T%d" % k: v for k, v in dl.items()},
        "downlink_note": "cdm_precode_batch (Algorithm 2, power scaling to rho/sqrt(C), rho = 1) on the same "
                         "channels, one 16-QAM symbol vector per (subcarrier, vector); paper's downlink Table I "
                         "cells for context",
    }
    out.setdefault("host", _host_info())
    print(json.dumps(out))


def _hbm_probes(cdm, dev, stream):
    """Achievable HBM rates on this device with the library's own kernels, each over a
    1 GiB buffer, 5 timed launches after 2 untimed ones: a read-only stream (the ceiling
    the read-dominated sweep kernels are compared with) and a plain copy (read + write
    counted; its HBM counter readings calibrate FETCH_SIZE / WRITE_SIZE).  GB/s."""
    import torch
    nb = 1 << 30
    src = torch.empty(nb // 16, dtype=torch.complex128, device=dev)
    dst = torch.empty_like(src)
    acc = torch.empty((cdm.STREAM_READ_SLOTS, 4), dtype=torch.int32, device=dev)

    def rate(fn, moved):
        for _ in range(2):
            fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(5):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return moved * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9

    out = {"read_gbs": rate(lambda: cdm.stream_read(src, acc), nb),
           "copy_gbs": rate(lambda: cdm.stream_copy(src, dst), 2 * nb)}
    del src, dst, acc
    return out


def _ceiling(achieved, probes):
    """The roofline's measured-ceiling fields: the probes and the fraction of the
    read-only rate that the kernel reaches."""
    return {"measured_read_gbs": probes["read_gbs"], "measured_copy_gbs": probes["copy_gbs"],
            "frac_of_measured_read": achieved / probes["read_gbs"]}


def _graph(fn):
    """Capture fn() (already run once eagerly on the capture stream) in a HIP graph."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return g


def _time_graph(g, steps, warmup):
    import torch
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def bench_warm(a):
    """Learned warm start on the uneven-batch distribution (m ~ U{64..2048}, n = m/2,
    complex128, lambda 0.1).  Training: `--train` instances (seeds 1,000,000 + j, in
    chunks of 4096) solved to a relative step of 1e-11; per-coordinate features and
    solutions train the 8 -> 512 -> 512 -> 2 network.  Held out: 4096 instances (seeds
    0..4095) solved to a relative step of 1e-8 from x0 = 0 (cold) and from the
    network's x0 (warm: feature pass + network + solve, all in one HIP graph), both with
    plain complex128 sweeps and with the mixed-precision refinement; `value` is the warm
    mixed-precision form."""
    import torch

    from paper_1902_08653_amd import cdm, inputs
    from paper_1902_08653_amd.warmstart import WarmStart
    dev = torch.device("cuda:0")
    c128 = torch.complex128
    tol, eps = 1e-8, 1e-6
    log = lambda msg: print("[bench] " + msg, file=sys.stderr, flush=True)
    # ---- training data ----------------------------------------------------------
    t0 = time.time()
    Fs, Ts, gen_ms = [], [], 0.0
    for c0 in range(0, a.train, 4096):
        cnt = min(4096, a.train - c0)
        H, y, m, n = inputs.batch_uneven_device(cnt, seed0=1_000_000 + c0, dtype=c128, device=dev)
        p = cdm.BatchedPlan(m, n, precision="c128", T_max=500, tol=1e-11)
        xs, _ = p.solve(H, y, N0=a.lam)
        F, T = WarmStart.training_rows(p, H, y, xs, N0=a.lam)
        Fs.append(F)
        Ts.append(T)
        p.close()
        del H, y, xs
    F = torch.cat(Fs)
    T = torch.cat(Ts)
    del Fs, Ts
    torch.cuda.synchronize()
    log("training rows %d from %d instances in %.1f s" % (F.shape[0], a.train, time.time() - t0))
    ws = WarmStart(hidden=512, max_rows=1 << 18, seed=0)
    t0 = time.time()
    hist = ws.fit(F, T, epochs=a.epochs, batch=16384, lr=1e-3, seed=0, log=log)
    torch.cuda.synchronize()
    train_s = time.time() - t0
    train_rows = int(F.shape[0])
    steps_per_epoch = (train_rows + 16383) // 16384
    train_flop = a.epochs * 3 * 2.0 * F.shape[0] * (8 * 512 + 512 * 512 + 512 * 2)
    zs = F[:, :2].double()
    lin_a = float((zs * T.double()).sum() / (zs * zs).sum())   # best real shrinkage of z, for context
    lin_mse = float(((T.double() - lin_a * zs) ** 2).mean())
    del F, T, zs
    # ---- held-out comparison ---------------------------------------------------------
    # four forms on the same batch, each one HIP graph: plain complex128 sweeps and the
    # mixed-precision refinement (complex64 or BF16 inner copy), each cold (x0 = 0) and
    # warm (feature pass + network + solve)
    H, y, m, n = inputs.batch_uneven_device(a.batch, seed0=0, dtype=c128, device=dev)
    inner = {"c64": "mixed-c64", "bf16": "bf16"}[a.inner]
    plans = {"plain": cdm.BatchedPlan(m, n, precision="c128", T_max=500, tol=tol, autotune=True),
             "mixed": cdm.BatchedPlan(m, n, precision=inner, T_max=8 if a.inner == "c64" else 16, tol=tol,
                                      autotune=True)}
    N = int(n.astype(np.int64).sum())
    x0 = torch.empty(N, dtype=c128, device=dev)
    Fh = torch.empty((N, 8), dtype=torch.float32, device=dev)
    xs = {k: torch.empty(N, dtype=c128, device=dev) for k in ("plain_cold", "plain_warm", "mixed_cold", "mixed_warm")}
    infos = {k: torch.empty(32 * a.batch, dtype=torch.uint8, device=dev) for k in xs}

    def form(name):
        plan = plans[name.split("_")[0]]
        if name.endswith("cold"):
            return lambda: plan.solve(H, y, N0=a.lam, x=xs[name], info=infos[name])
        return lambda: ws.solve(plan, H, y, N0=a.lam, x0=x0, feat=Fh, x=xs[name], info=infos[name])

    ms = {}
    for k in xs:
        g = _graph(form(k))
        ms[k] = _time_graph(g, a.steps, a.warmup)
        del g
    # stage split of the warm mixed form (eager, events on the current stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    plans["mixed"].features(H, y, N0=a.lam, out=Fh)
    ev[1].record()
    ws.net.predict(Fh, c128, out=x0)
    ev[2].record()
    plans["mixed"].solve(H, y, N0=a.lam, x0=x0, x=xs["mixed_warm"], info=infos["mixed_warm"])
    ev[3].record()
    torch.cuda.synchronize()
    st = [ev[i].elapsed_time(ev[i + 1]) for i in range(3)]
    rec = {k: cdm.parse_info(v) for k, v in infos.items()}
    mn = m.astype(np.int64) * n.astype(np.int64)
    lowsz = 8 if a.inner == "c64" else 4

    def stats(k):
        r = rec[k]
        d = {"ms": ms[k], "instance_solves_per_s": a.batch * 1000.0 / ms[k],
             "flags_or": int(np.bitwise_or.reduce(r["flags"]))}
        if k.startswith("plain"):
            d["sweeps_mean"] = float(r["sweeps"].mean())
        else:
            d["outer_mean"] = float(r["sweeps"].mean())
            d["inner_sweeps_mean"] = float(r["reserved"].mean())
        return d

    for k in ms:
        log("%s: %.2f ms %s" % (k, ms[k], {q: v for q, v in stats(k).items() if q != "ms"}))
    # algorithmic bytes of the mixed kernel per instance: complex128 passes (the first
    # step of a cold start needs only g), inner sweeps over the copy, the copy's write
    rm = rec["mixed_warm"]
    passes = 2 * rm["sweeps"].astype(np.int64)
    mixed_bytes = float((mn * (16 * passes + lowsz * rm["reserved"].astype(np.int64) + lowsz)).sum())
    mlp_flop = 2.0 * N * (8 * 512 + 512 * 512 + 512 * 2)
    cpu, errs = None, []
    if not a.no_oracle:
        from oracle import oracle
        oracle.build()
        order = np.argsort(-mn)
        pick = order[np.linspace(0, a.batch - 1, a.sample or 12).astype(int)]
        ho = np.concatenate([[0], np.cumsum(mn)[:-1]])
        yo = np.concatenate([[0], np.cumsum(m.astype(np.int64))[:-1]])
        xo = np.concatenate([[0], np.cumsum(n.astype(np.int64))[:-1]])
        xg = {k: v.cpu().numpy() for k, v in xs.items()}
        cpu_s, cpu_bytes = 0.0, 0.0
        for i in pick:
            Hi = H[ho[i]:ho[i] + m[i] * n[i]].cpu().numpy().reshape(n[i], m[i]).T
            yi = y[yo[i]:yo[i] + m[i]].cpu().numpy()
            tc = time.perf_counter()
            ref = oracle.local_cd(Hi, yi, a.lam, T_max=500, tol=tol)
            cpu_s += time.perf_counter() - tc
            cpu_bytes += ref["sweeps"] * float(mn[i] * 16)
            exact = oracle.local_cd(Hi, yi, a.lam, T_max=2000, tol=1e-13)["x"]
            nr = np.linalg.norm(exact)
            sl = slice(xo[i], xo[i] + n[i])
            errs.append(max(np.linalg.norm(v[sl] - exact) for v in xg.values()) / nr)
        full = float((rec["plain_cold"]["sweeps"].astype(np.int64) * mn * 16).sum())
        cpu = {"value": a.batch / (cpu_s * full / cpu_bytes), "unit": "instance solves/s", "cores": 1,
               "kind": "oracle",
               "sample": "%d held-out instances spread over the size range, cold oracle to rel. step %g "
                         "on one thread (%.1f s), scaled by the batch's sweep-weighted H bytes"
                         % (len(pick), tol, cpu_s)}
    achieved = mixed_bytes / (st[2] * 1e-3) / 1e9
    out = {
        "metric": "solves/sec to fixed rel. tolerance vs FP64 oracle",
        "value": a.batch * 1000.0 / ms["mixed_warm"],
        "unit": "instance solves/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms["mixed_warm"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if a.inner == "c64" else "bf16+f32+f64",
        "data": "synthetic",
        "config": {"workload": "warm-started mixed-precision batched solve: %d held-out uneven uplink instances, "
                               "m~U{64..2048}, n=m/2, complex128 data, lambda=%g, rel. tol %g; network "
                               "8-512-512-2 trained on %d instances (%d epochs); inner copy %s"
                               % (a.batch, a.lam, tol, a.train, a.epochs, a.inner),
                   "engine": json.loads(plans["mixed"].describe())},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_cd_wg_mixed (warm solve)",
                     "algorithmic_bytes_per_launch": mixed_bytes, "avg_launch_ms": st[2]},
        "cpu_baseline": cpu,
        "forms": {k: stats(k) for k in ms},
        "speedup_vs_plain_cold": {k: ms["plain_cold"] / ms[k] for k in ms},
        # the two effects apart: the learned warm start against the same form cold (> 1:
        # the network pays for itself), and mixed precision against plain, both cold
        "network_net_effect": {"plain": ms["plain_cold"] / ms["plain_warm"],
                               "mixed": ms["mixed_cold"] / ms["mixed_warm"]},
        "mixed_precision_effect_cold": ms["plain_cold"] / ms["mixed_cold"],
        "warm_stage_ms": {"features": st[0], "network": st[1], "solve": st[2]},
        "network_tflops": mlp_flop / (st[1] * 1e-3) / 1e12,
        "train": {"rows": train_rows, "steps": a.epochs * steps_per_epoch, "seconds": train_s,
                  "tflops": train_flop / train_s / 1e12, "loss_per_epoch": hist,
                  "linear_shrinkage_mse": lin_mse},
        "accuracy": {"max_rel_err_vs_oracle_sample": max(errs) if errs else None, "eps": eps,
                     "within_eps": bool(max(errs) <= eps) if errs else None},
    }
    out.setdefault("host", _host_info())
    print(json.dumps(out))
    for pl in plans.values():
        pl.close()
    ws.close()


if __name__ == "__main__":
    main()
