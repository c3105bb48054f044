#!/usr/bin/env python3
"""Benchmark of the FFT-based block lower-triangular Toeplitz matvec on one MI355X.

Workload: the paper's single-GPU shape Nt=1000, Nd=100, Nm=5000 (Section
4.1.2), F blocks iid N(0,1)/sqrt(Nm) * exp(-t/200), m and d iid N(0,1),
seeded.  One step = one forward matvec F m plus one adjoint matvec F^T d in
float64, inputs resident in HBM.  ``value`` is float64 matvecs per second.

Besides the JSON fields of the benchmark contract the line carries:
  roofline      the dominant kernel (the float64 forward product), its
                algorithmic bytes per launch over its average duration from
                HIP events recorded by the library on the launch stream
  cpu_baseline  the float64 CPU oracle timed on this host (one forward and one
                adjoint at the full shape)
  kernels_ms    average per-kernel times of both directions
  rel_err       float64 relative L2 error of both directions vs the oracle
  mixed         per-phase mixed precision: time and error per configuration,
                the Pareto front and the fastest configuration under each tolerance
  multi_rhs     64 right-hand sides through the matrix-core products
  serving       the continuous-batching server under Poisson load
  sbgemv        the standalone strided-batched product at short-wide shapes
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "matvecs/s + HBM GB/s at N_t=1000,N_d=100,N_m=5000; FP64 vs mixed @rel err"
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemv_fwd_f64_paper_traffic.json")
# sources the product kernels are compiled from (the counters go stale when any changes)
GEMV_SRCS = [os.path.join(ROOT, "paper_2508_10202_amd", "csrc", f)
             for f in ("ftm_gemv.hip", "ftm_device.h", "ftm_kernels.h")]

# configurations timed by default: the paper's 32 {d,s} assignments plus
# half-precision storage variants (all in execution order pad,fft,gemv,ifft,unpad)
HALF_CONFIGS = ["ddhdd", "ddbdd", "dhhhd", "dbbbd", "hhhhh", "bbbbb", "dshsd", "dsbsd", "ddsdd+a64"]


def ds_configs():
    out = []
    for i in range(32):
        out.append("".join("s" if (i >> (4 - j)) & 1 else "d" for j in range(5)))
    return out


def all_configs():
    import itertools
    out = ["".join(c) for c in itertools.product("dshb", repeat=5)]
    return out + [c + "+a64" for c in out if c[2] == "s"]


def gemv_bytes(s, fbytes: int, vbytes: int = 16) -> float:
    """Algorithmic bytes of one product launch: the spectrum once, the
    transformed input read once, the transformed output written once."""
    return s.K * s.Nd * s.Nm * fbytes + s.K * (s.Nm + s.Nd) * vbytes


def matvec_bytes(s, fbytes: int) -> float:
    """Algorithmic bytes of one whole matvec: spectrum + float64 input + float64 output."""
    return s.K * s.Nd * s.Nm * fbytes + s.Nt * (s.Nm + s.Nd) * 8


def pareto(rows):
    """Rows not dominated in (time, error): nothing at least as good in both and better in one."""
    front = []
    for r in rows:
        dom = any((q["ms"] <= r["ms"] and q["err"] <= r["err"]) and (q["ms"] < r["ms"] or q["err"] < r["err"])
                  for q in rows)
        if not dom:
            front.append(r["prec"])
    return front


def gemv_source_sha256():
    h = hashlib.sha256()
    for f in GEMV_SRCS:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_record():
    """HBM traffic of the dominant kernel from committed PMC counter runs, if
    they were taken on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    sha = gemv_source_sha256()
    if rec.get("kernel_source_sha256") != sha:
        return None
    return rec.get("bytes_per_launch")


# unit roundoffs of the storage formats
UNIT = {"d": 2.0 ** -53, "s": 2.0 ** -24, "h": 2.0 ** -11, "b": 2.0 ** -8}


def error_window(prec: str, L: int, n: int):
    """Window an assignment's relative error must fall in, shaped after the
    paper's eq. (error) with unit constants: pad and unpad rounding once, the
    transforms growing like log2 L, the product's rounding of the spectrum and
    of its input, its accumulation (log2 n terms, n = Nm forward, Nd adjoint)
    and the float64 setup transform.  Upper edge 4x that budget; lower edge the
    largest unit roundoff present / 64 (a phase that skipped its rounding)."""
    body, _, acc = prec.partition("+")
    acc_fmt = ("d" if acc == "a64" else "s") if acc else ("d" if body[2] == "d" else "s")
    lg = math.log2(L)
    budget = (UNIT[body[0]] + UNIT[body[1]] * lg + 2 * UNIT[body[2]] + UNIT[acc_fmt] * math.log2(max(n, 2))
              + UNIT[body[3]] * lg + UNIT[body[4]] + UNIT["d"] * lg)
    lo = max(UNIT[c] for c in body) / 64 if body != "ddddd" else 0.0
    return lo, 4 * budget + 1e-14


def best_under(rows, base_ms, tols=(1e-12, 1e-7, 1e-6, 1e-3, 1e-2)):
    out = {}
    for tol in tols:
        ok = [r for r in rows if r["err"] <= tol]
        if ok:
            b = min(ok, key=lambda r: (r["ms"], r["err"]))
            out[f"{tol:g}"] = {"prec": b["prec"], "ms": b["ms"], "err": b["err"],
                               "speedup_vs_fp64": round(base_ms / b["ms"], 3)}
    return out


def mixed_section(log, op, s, mt, dt, dout, mout, ref_d, ref_m, confs, reps=5):
    """Every configuration in ``confs`` timed in both directions at the paper's
    shape: per-kernel times from the library's events (reps calls after one
    warm call), relative L2 error against the oracle output (computed once on
    the CPU, compared on the device), and whether the error lies in its
    eq. (error) window."""
    import torch
    dev = mt.device
    refs = {"fwd": torch.from_numpy(ref_d).to(dev), "adj": torch.from_numpy(ref_m).to(dev)}
    ref_norm = {k: float(torch.linalg.vector_norm(v)) for k, v in refs.items()}
    rows = {"fwd": [], "adj": []}
    t0 = time.time()
    for i, c in enumerate(confs):
        op.set_precision(fwd=c, adj=c)
        for name, fn, x, out in (("fwd", op.matvec, mt, dout), ("adj", op.rmatvec, dt, mout)):
            fn(x, out=out)
            op.profile(True)
            for _ in range(reps):
                fn(x, out=out)
            p = op.profile_read()
            op.profile(False)
            kms = p[name]
            err = float(torch.linalg.vector_norm(out - refs[name])) / ref_norm[name]
            lo, hi = error_window(c, s.L, s.Nm if name == "fwd" else s.Nd)
            rows[name].append({"prec": c, "ms": round(sum(kms), 5), "kernels_ms": [round(v, 5) for v in kms],
                               "err": float(f"{err:.4e}"), "in_window": bool(lo <= err <= hi)})
        if (i + 1) % 128 == 0:
            log(f"mixed: {i + 1}/{len(confs)} configurations in {time.time() - t0:.0f}s")
    op.set_precision(fwd="ddddd", adj="ddddd")
    ds = set(ds_configs())
    mixed = {"n_configs": len(confs), "reps": reps, "configs": rows, "pareto": {}, "best": {},
             "out_of_window": {}, "ds_subset": {"pareto": {}, "best": {}}}
    for k, v in rows.items():
        base = next(r for r in v if r["prec"] == "ddddd")["ms"]
        mixed["pareto"][k] = pareto(v)
        mixed["best"][k] = best_under(v, base)
        mixed["out_of_window"][k] = [r["prec"] for r in v if not r["in_window"]]
        sub = [r for r in v if r["prec"] in ds]
        mixed["ds_subset"]["pareto"][k] = pareto(sub)
        mixed["ds_subset"]["best"][k] = best_under(sub, base)
    log("mixed best: " + json.dumps(mixed["best"]))
    log("mixed out of window: " + json.dumps(mixed["out_of_window"]))
    return mixed


PEAK_FP32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP64_TFLOPS = 78.6


def multi_rhs_section(log, products_only=False):
    """64 right-hand sides at Nt=512, Nd=128, Nm=4096: the per-frequency product
    on the matrix cores (FP32 and BF16 storage, FP32 accumulation) against 64
    separate float64 matvecs on the same GPU; four right-hand sides are checked
    against the oracle.  Then the nrhs sweep and the Hessian assembly, unless
    `products_only`."""
    import torch

    import oracle
    from paper_2508_10202_amd import Operator
    from workloads import MULTI_RHS_NRHS, config_inputs
    s, F, M, D = config_inputs("multi_rhs", nrhs=MULTI_RHS_NRHS)
    B = MULTI_RHS_NRHS
    dev = torch.device("cuda:0")
    op = Operator(torch.from_numpy(F).to(dev), spectra=("s", "b"), max_rhs=B)
    Mt, Dt = torch.from_numpy(M).to(dev), torch.from_numpy(D).to(dev)
    Yd = torch.empty((B, s.Nt, s.Nd), dtype=torch.float64, device=dev)
    Ym = torch.empty((B, s.Nt, s.Nm), dtype=torch.float64, device=dev)
    pick = [0, 21, 42, 63]
    ref_d, ref_m = oracle.forward(F, M[pick]), oracle.adjoint(F, D[pick])
    flops = 8.0 * s.K * s.Nd * s.Nm * B
    out = {"workload": f"Nt={s.Nt} Nd={s.Nd} Nm={s.Nm}, {B} right-hand sides", "flops_per_product": flops}

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        op.profile(True)
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        p = op.profile_read()
        op.profile(False)
        return p

    # baseline: 64 separate float64 matvecs per direction
    op.set_precision(fwd="ddddd", adj="ddddd")
    def sep():
        for b in range(B):
            op.matvec(Mt[b], out=Yd[b])
            op.rmatvec(Dt[b], out=Ym[b])
    p = timed(sep, reps=1)
    base_f, base_a = sum(p["fwd"]) * B, sum(p["adj"]) * B
    out["fp64_separate_ms"] = {"fwd": round(base_f, 3), "adj": round(base_a, 3)}
    for prec, peak, fbytes in (("ddsdd", PEAK_FP32_TFLOPS, 8), ("dbbbd", PEAK_BF16_TFLOPS, 4),
                               ("ddddd", PEAK_FP64_TFLOPS, 16), ("ddsdd+a64", PEAK_FP64_TFLOPS, 8)):
        op.set_precision(fwd=prec, adj=prec)
        p = timed(lambda: (op.matvec(Mt, out=Yd), op.rmatvec(Dt, out=Ym)))
        e_f = oracle.relative_l2(Yd[pick].cpu().numpy(), ref_d)
        e_a = oracle.relative_l2(Ym[pick].cpu().numpy(), ref_m)
        # bytes per complex entry of the product's input and output as the
        # library stores them (float64 between float64 phases, 16 bits for the
        # input of a half-precision product, float32 otherwise)
        body = prec.split("+")[0]
        xb = 16 if body[1] == body[2] == "d" else (4 if body[2] in "hb" else 8)
        yb = 16 if body[2] == body[3] == "d" else 8
        rec = {"peak_tflops": peak}
        for name, kms, err, base in (("fwd", p["fwd"], e_f, base_f), ("adj", p["adj"], e_a, base_a)):
            n_in, n_out = (s.Nd, s.Nm) if name == "adj" else (s.Nm, s.Nd)
            gemm_bytes = s.K * s.Nd * s.Nm * fbytes + s.K * B * (n_in * xb + n_out * yb)
            t = kms[1] * 1e-3
            rec[name] = {"kernels_ms": [round(x, 4) for x in kms], "matvec_ms": round(sum(kms), 4),
                         "gemm_tflops": round(flops / t / 1e12, 2), "mfma_frac": round(flops / t / 1e12 / peak, 4),
                         "gemm_gbs": round(gemm_bytes / t / 1e9, 1), "rel_err": float(f"{err:.3e}"),
                         "speedup_vs_fp64_separate": round(base / sum(kms), 2)}
        out[prec] = rec
        log(f"multi-rhs {prec}: " + json.dumps(rec))
    if not products_only:
        out["nrhs_sweep"] = {prec: nrhs_sweep(op, s, Mt, Dt, prec) for prec in ("ddsdd", "ddddd")}
        log("multi-rhs nrhs sweep: " + json.dumps(out["nrhs_sweep"]))
        out["hessian"] = hessian_section(log, op, F, s, "Nt=512 Nd=128 Nm=4096")
    op.close()
    return out


def nrhs_sweep(op, s, Mt, Dt, prec, counts=(1, 2, 4, 8, 16, 32, 64), reps=3):
    """Time per matvec of nrhs right-hand sides, per direction, with the
    automatic choice (the matrix-core GEMM from the crossover on) and with one
    matrix-vector product per vector; ``auto_le_gemv`` says whether the
    automatic choice was no slower (within 3%)."""
    import torch
    op.set_precision(fwd=prec, adj=prec)
    dev = Mt.device
    Yd = torch.empty((max(counts), s.Nt, s.Nd), dtype=torch.float64, device=dev)
    Ym = torch.empty((max(counts), s.Nt, s.Nm), dtype=torch.float64, device=dev)
    rows = []
    for n in counts:
        row = {"nrhs": n}
        for mode in ("auto", "gemv"):
            op.set_rhs_mode(mode)
            ms = []
            for fn, x, y in ((op.matvec, Mt, Yd), (op.rmatvec, Dt, Ym)):
                fn(x[:n], out=y[:n])
                ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                ev0.record()
                for _ in range(reps):
                    fn(x[:n], out=y[:n])
                ev1.record()
                torch.cuda.synchronize()
                ms.append(round(ev0.elapsed_time(ev1) / reps, 4))
            row[f"{mode}_ms"] = ms
        row["auto_le_gemv"] = all(a <= 1.03 * g for a, g in zip(row["auto_ms"], row["gemv_ms"]))
        rows.append(row)
    op.set_rhs_mode("auto")
    return rows


def hessian_section(log, op, F, s, label, batch=64, full_prec="ddsdd", sample_prec="ddddd", sample_batches=8):
    """Assembly of the dense data-space Hessian F F^T (identity prior, the
    outer-loop workload of Section 3.2): all Nd * Nt actions on the unit
    vectors, in batches through ftm_hessian_apply, at ``full_prec``; a timed
    sample of ``sample_batches`` batches at ``sample_prec``.  Columns are
    streamed through one output buffer (storing them is a pointer change).
    One column is checked against the oracle."""
    import numpy as np
    import torch

    import oracle
    dev = torch.device("cuda:0")
    n_act = s.Nt * s.Nd
    X = torch.zeros((batch, s.Nt, s.Nd), dtype=torch.float64, device=dev)
    Y = torch.empty_like(X)
    Xf = X.view(batch, -1)
    ar = torch.arange(batch, device=dev)
    out = {"workload": f"{label}: {n_act} actions F F^T e_j in batches of {batch}"}
    for prec, nb in ((full_prec, (n_act + batch - 1) // batch), (sample_prec, sample_batches)):
        op.set_precision(fwd=prec, adj=prec)
        ws = torch.empty(((op.hessian_workspace_size(batch) + 7) // 8,), dtype=torch.float64, device=dev)
        X.zero_()                                   # no unit entries left from the previous pass
        op.hessian(X, workspace=ws, out=Y)          # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prev = None
        for i in range(nb):
            j = (i * batch + ar) % n_act
            if prev is not None:
                Xf[ar, prev] = 0.0
            Xf[ar, j] = 1.0
            prev = j
            op.hessian(X, workspace=ws, out=Y)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        # the last batch's first column against the oracle
        jcol = int(prev[0])
        e = np.zeros((s.Nt, s.Nd))
        e.flat[jcol] = 1.0
        err = oracle.relative_l2(Y[0].cpu().numpy(), oracle.hessian_data_space(F, e))
        rec = {"actions": nb * batch, "seconds": round(dt, 3), "actions_per_s": round(nb * batch / dt, 1),
               "ms_per_batch": round(dt / nb * 1e3, 3), "rel_err_sampled_column": float(f"{err:.3e}"),
               "projected_full_assembly_s": round(n_act / (nb * batch / dt), 2)}
        out[prec] = rec
        log(f"hessian {label} {prec}: " + json.dumps(rec))
        del ws
    return out


def sbgemv_section(log):
    """The standalone strided-batched product at the shapes of the paper's
    kernel benchmark (Section 4.1.1): batch 100, short-wide m x n matrices
    with n = 4096 and m from 32 to 4096, transposed for real types and
    conjugate-transposed for complex ones; also op N at m = 128.  GB/s counts
    the matrices, x and y once; sampled batch entries are checked against the
    oracle at m = 128."""
    import torch

    import oracle
    from paper_2508_10202_amd import sbgemv
    dev = torch.device("cuda:0")
    types = (("s", torch.float32, "T"), ("d", torch.float64, "T"), ("c", torch.complex64, "C"),
             ("z", torch.complex128, "C"))
    batch, n = 100, 4096
    g = torch.Generator(device=dev).manual_seed(2508_10202 + 600)
    rows = []
    for t, dt, op0 in types:
        for m, op in ((32, op0), (128, op0), (1024, op0), (4096, op0), (128, "N")):
            A = torch.randn((batch, n, m), dtype=dt, device=dev, generator=g)
            nx, ny = (n, m) if op == "N" else (m, n)
            x = torch.randn((batch, nx), dtype=dt, device=dev, generator=g)
            y = torch.empty((batch, ny), dtype=dt, device=dev)
            for _ in range(3):
                sbgemv(A, x, op=op, y=y)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps, trials = 20, []
            for _ in range(3):
                # keep the GPU busy while the host enqueues the timed launches, so
                # that host-side call overhead never leaves the GPU idle between them
                torch.cuda._sleep(5_000_000)
                e0.record()
                for _ in range(reps):
                    sbgemv(A, x, op=op, y=y)
                e1.record()
                torch.cuda.synchronize()
                trials.append(e0.elapsed_time(e1) / reps)
            ms = sorted(trials)[1]                     # median of 3 trials of 20 launches
            nbytes = batch * (m * n + m + n) * A.element_size()
            row = {"type": t, "op": op, "m": m, "n": n, "batch": batch, "ms": round(ms, 4),
                   "trials_ms": [round(v, 4) for v in trials],
                   "gbs": round(nbytes / ms / 1e6, 1), "frac": round(nbytes / ms / 1e6 / PEAK_HBM_GBS, 3)}
            if m == 128:
                pick = [0, 99]
                ref = oracle.sbgemv(op, A[pick].cpu().numpy(), m, x[pick].cpu().numpy())
                row["rel_err"] = float(f"{oracle.relative_l2(y[pick].cpu().numpy(), ref):.3e}")
            rows.append(row)
            del A, x, y
    torch.cuda.empty_cache()
    log("sbgemv: " + json.dumps(rows))
    return rows


def serving_section(log, seconds: float, warmup: float = 1.0, rate: float = 2000.0, budget_gib: float = 16.0):
    """Poisson arrivals at `rate` req/s against 4 device-resident FP32
    operators; each request is forward or adjoint (50/50) with 1..32 vectors,
    operator uniform.  Workspace budget `budget_gib` (16 GiB by default; at
    4 GiB it binds: a 32-vector request on the largest operators needs 1.3-2.1
    GB, and a coalesced 64-vector batch twice that).  A second,
    shorter run offers the same mix at 3/4 of the throughput the first one
    reached (`below_capacity`), where the latency is not dominated by
    queueing.  `capacity` is what the GPU can serve with one batch at a time:
    each operator and direction timed alone on 16 vectors (about one mean
    request) and on 64 (a full coalesced batch), averaged over the uniform
    mix of operators and directions."""
    import numpy as np
    import torch

    import oracle
    from paper_2508_10202_amd import Operator, Server
    from workloads import SERVING_OPS, make_F, seed_for

    dev = torch.device("cuda:0")
    ops, Fs = [], []
    for i, sh in enumerate(SERVING_OPS):
        F = make_F(sh, seed_for(5, 10 + i))
        Fs.append(F if i in (0, 1) else None)         # host copies kept for the sampled checks
        ops.append(Operator(torch.from_numpy(F).to(dev), fwd="sssss", adj="sssss", spectra=("s",)))
        del F
    torch.cuda.synchronize()
    # input pools: 2 per (operator, direction), 32 vectors each, iid N(0,1) (seeded)
    g = torch.Generator(device=dev).manual_seed(seed_for(5, 3))
    pools = {}
    for i, op in enumerate(ops):
        for adj in (0, 1):
            n = op.Nd if adj else op.Nm
            pools[i, adj] = [torch.randn((32, op.Nt, n), dtype=torch.float64, device=dev, generator=g)
                             for _ in range(2)]
    torch.cuda.synchronize()
    # serial capacity: ms per batch of 16 and of 64 vectors, per (operator, direction)
    cap = {}
    wsb = max(op.workspace_size(64, adjoint=bool(a)) for op in ops for a in (0, 1))
    cws = torch.empty(((wsb + 7) // 8,), dtype=torch.float64, device=dev)
    for i, op in enumerate(ops):
        for adj in (0, 1):
            n = op.Nd if adj else op.Nm
            xin = torch.randn((64, op.Nt, n), dtype=torch.float64, device=dev, generator=g)
            yout = torch.empty((64, op.Nt, op.Nm if adj else op.Nd), dtype=torch.float64, device=dev)
            for nb in (16, 64):
                def fn():
                    op.apply(xin[:nb], cws, adjoint=bool(adj), out=yout[:nb])
                fn()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(5):
                    fn()
                torch.cuda.synchronize()
                cap[i, adj, nb] = (time.perf_counter() - t0) / 5 * 1e3
            del xin, yout
    del cws
    mean_vec = 16.5                                   # mean of 1..32 vectors per request
    ms16 = float(np.mean([cap[i, a, 16] for i in range(len(ops)) for a in (0, 1)])) * mean_vec / 16
    ms64 = float(np.mean([cap[i, a, 64] for i in range(len(ops)) for a in (0, 1)])) * mean_vec / 64
    capacity = {"ms_per_batch": {f"op{i}_{'adj' if a else 'fwd'}_{nb}": round(v, 3) for (i, a, nb), v in cap.items()},
                "req_s_at_16_vector_batches": round(1e3 / ms16, 1), "req_s_at_64_vector_batches": round(1e3 / ms64, 1)}
    log("serving capacity: " + json.dumps({k: v for k, v in capacity.items() if k != "ms_per_batch"}))
    budget = int(budget_gib * (1 << 30)) // 256 * 256
    # output buffers: a ring of 16 per (operator, direction), 32 vectors each; a
    # buffer is reused once the request that wrote it has completed (if it has
    # not, the client waits: that delay counts against the request's latency,
    # which is measured from its scheduled arrival)
    ring = 16
    outs = {}
    for i, op in enumerate(ops):
        for adj in (0, 1):
            n = op.Nm if adj else op.Nd
            outs[i, adj] = [torch.empty((32, op.Nt, n), dtype=torch.float64, device=dev) for _ in range(ring)]

    def run(rate, seconds, stream, keep_samples):
        rng = np.random.default_rng(seed_for(5, stream))
        total = warmup + seconds
        n_req = int(rate * total * 1.2) + 16
        arrivals = np.cumsum(rng.exponential(1.0 / rate, n_req))
        arrivals = arrivals[arrivals < total]
        kinds = rng.integers(0, len(ops), len(arrivals))
        dirs = rng.integers(0, 2, len(arrivals))
        nrhs = rng.integers(1, 33, len(arrivals))
        srv = Server(workspace_budget=budget, n_slots=4, max_batch_rhs=64)
        owner = {}
        counters = {key: 0 for key in outs}
        tickets, keep, t_sub = [], {}, np.empty(len(arrivals))
        sample = set(range(0, len(arrivals), max(1, len(arrivals) // 8))) if keep_samples else set()
        t0 = time.perf_counter()
        for i, (ta, k, a, nr) in enumerate(zip(arrivals, kinds, dirs, nrhs)):
            key = (int(k), int(a))
            slot = counters[key] % ring
            counters[key] += 1
            prev = owner.get((key, slot))
            if prev is not None:
                srv.wait(prev, timeout=120)
            while time.perf_counter() - t0 < ta:
                pass
            x = pools[key][i % 2][: int(nr)]
            y = outs[key][slot][: int(nr)]
            t_sub[i] = time.perf_counter() - t0
            t, _ = srv.submit(ops[key[0]], x, adjoint=bool(a), out=y)
            owner[(key, slot)] = t
            tickets.append(t)
            if i in sample and key[0] in (0, 1):
                srv.wait(t, timeout=120)
                keep[i] = (t, y.clone(), k, a, nr)
        for t in tickets:
            srv.wait(t, timeout=120)
        t_end = time.perf_counter() - t0
        lat = srv.latencies(tickets[0], len(tickets))
        lag = t_sub - arrivals                      # client-side delay before submit
        st = srv.stats()
        measured = arrivals >= warmup
        lm = lat[measured] * 1e3
        la = (lat + lag)[measured] * 1e3            # from the scheduled arrival
        n_meas = int(measured.sum())
        vec = int(nrhs[measured].sum())
        rec = {"workload": "4 FP32 operators (Nt,Nd,Nm) = " + ", ".join(f"({s.Nt},{s.Nd},{s.Nm})" for s in SERVING_OPS)
                           + f"; Poisson {rate:g} req/s; forward/adjoint 50/50; 1-32 vectors uniform; {seconds:g} s "
                           + f"measured after {warmup:g} s warm-up",
               "requests": n_meas, "p50_ms": round(float(np.percentile(la, 50)), 3),
               "p99_ms": round(float(np.percentile(la, 99)), 3), "mean_ms": round(float(la.mean()), 3),
               "server_p50_ms": round(float(np.percentile(lm, 50)), 3),
               "server_p99_ms": round(float(np.percentile(lm, 99)), 3),
               "throughput_req_s": round(n_meas / max(t_end - warmup, 1e-9), 1),
               "vectors_s": round(vec / max(t_end - warmup, 1e-9), 1),
               "offered_req_s": round(rate, 1), "wall_s": round(t_end, 2),
               "max_submit_lag_ms": round(float(lag.max() * 1e3), 3),
               "workspace_budget_bytes": budget, "capacity": capacity, "stats": st}
        return rec, srv, keep

    out, srv, keep = run(rate, seconds, 4, True)
    # the same request alone on an idle server equals its result in the mix
    diffs = []
    for i, (t, y, k, a, nr) in keep.items():
        k, a, nr = int(k), int(a), int(nr)
        x = pools[k, a][i % 2][:nr]
        t2, y2 = srv.submit(ops[k], x, adjoint=bool(a))
        srv.wait(t2, timeout=60)
        xh = x.cpu().numpy()
        ref = oracle.adjoint(Fs[k], xh) if a else oracle.forward(Fs[k], xh)
        diffs.append({"request": i, "op": k, "adjoint": a, "nrhs": nr,
                      "mix_vs_alone": float(f"{oracle.relative_l2(y.cpu().numpy(), y2.cpu().numpy()):.3e}"),
                      "mix_vs_oracle": float(f"{oracle.relative_l2(y.cpu().numpy(), ref):.3e}")})
    out["sampled_checks"] = diffs
    srv.close()
    # the same mix offered below the capacity just measured: latency without
    # the unbounded queueing of an overloaded server
    below, srv2, _ = run(max(50.0, 0.75 * out["throughput_req_s"]), max(2.0, seconds / 2), 6, False)
    srv2.close()
    out["below_capacity"] = {k: v for k, v in below.items() if k != "workspace_budget_bytes"}
    log("serving below capacity: " + json.dumps({k: v for k, v in below.items() if k != "stats"}))
    out["small_requests"] = small_request_latency(ops[:2], pools, Server, budget)
    log("serving small requests: " + json.dumps(out["small_requests"]))
    for op in ops:
        op.close()
    log("serving: " + json.dumps({k: v for k, v in out.items() if k not in ("sampled_checks", "stats")}))
    return out


def small_request_latency(ops, pools, Server, budget, reps=50):
    """One-vector requests on the two small serving operators, one at a time:
    the median latency of a direct call (launch + synchronize), of a replayed
    HIP graph of the same call, and of a server round trip (submit + wait on
    an idle server, measured by the client), beside the GPU time of the
    call's three kernels.  The difference is launch and notification
    overhead."""
    import statistics

    import torch
    rows = []
    srv = Server(workspace_budget=budget, n_slots=4, max_batch_rhs=64)
    for i, op in enumerate(ops):
        for adj in (0, 1):
            x = pools[i, adj][0][:1]
            y = torch.empty((1, op.Nt, op.Nm if adj else op.Nd), dtype=torch.float64, device=x.device)
            fn = op.rmatvec if adj else op.matvec
            fn(x, out=y)
            op.profile(True)
            for _ in range(10):
                fn(x, out=y)
            torch.cuda.synchronize()
            gpu_us = sum(op.profile_read()["adj" if adj else "fwd"]) * 1e3
            op.profile(False)

            def med(call):
                lat = []
                for _ in range(reps):
                    t0 = time.perf_counter()
                    call()
                    lat.append(time.perf_counter() - t0)
                return round(statistics.median(lat) * 1e6, 1)

            direct = med(lambda: (fn(x, out=y), torch.cuda.synchronize()))
            g = op.graph(x, adjoint=bool(adj))
            graph = med(lambda: (g.launch(), torch.cuda.synchronize()))
            g.close()
            server = med(lambda: srv.wait(srv.submit(op, x, adjoint=bool(adj), out=y)[0], timeout=60))
            rows.append({"op": [op.Nt, op.Nd, op.Nm], "adjoint": adj, "kernels_us": round(gpu_us, 1),
                         "direct_us": direct, "graph_us": graph, "server_us": server})
    srv.close()
    return {"workload": "1-vector FP32 requests, one at a time, median of " + str(reps), "rows": rows}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--mixed", choices=["none", "subset", "all"], default="all",
                    help="mixed-precision configurations to time: every {d,s,h,b}^5 assignment plus the "
                         "float64-accumulated float32 products (all), or the 32 {d,s} ones plus 9 others (subset)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle", action="store_true",
                    help="skip the CPU oracle (no errors, no CPU baseline): for profiler runs")
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="after the timed work, copy a buffer of this size 3 times (device to device) "
                         "so HBM byte counters can be scaled against a plain copy of known size")
    ap.add_argument("--no-multi-rhs", action="store_true",
                    help="skip the 64-right-hand-side GEMM measurement (Nt=512, Nd=128, Nm=4096)")
    ap.add_argument("--multi-rhs-products-only", action="store_true",
                    help="of the many-right-hand-side sections run only the 64-vector products at "
                         "Nt=512, Nd=128, Nm=4096 (no nrhs sweeps, Hessian or standalone SBGEMV): for profiler runs")
    ap.add_argument("--serving-seconds", type=float, default=10.0,
                    help="measured duration of the serving run (after a 1 s warm-up); 0 skips it")
    ap.add_argument("--serving-budget-gib", type=float, default=16.0,
                    help="workspace budget of the serving run's server (16 GiB of the 288 GB)")
    ap.add_argument("--json-out", default=None, help="also write the full record here")
    args = ap.parse_args()
    if args.no_oracle:
        args.mixed = "none"
        args.no_cpu_baseline = True
        args.no_multi_rhs = True
        args.serving_seconds = 0.0

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the distributed "
              "layout is described, not built", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2508_10202_amd import Operator
    from workloads import config_inputs

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    t0 = time.time()
    s, F, m, d = config_inputs("paper")
    m, d = m[0], d[0]
    log(f"inputs generated in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    # the FP32 copy serves the multi-RHS sweep and the Hessian section; the
    # half copies serve the mixed-precision sweep
    spectra = (() if args.no_multi_rhs else ("s",)) if args.mixed == "none" else ("s", "h", "b")
    Ft = torch.from_numpy(F).to(dev)
    op = Operator(Ft, spectra=spectra, max_rhs=64)
    torch.cuda.synchronize()
    del Ft
    torch.cuda.empty_cache()
    log(f"operator ready ({op.device_bytes() / 1e9:.2f} GB on device)")
    mt, dt = torch.from_numpy(m).to(dev), torch.from_numpy(d).to(dev)
    dout = torch.empty((s.Nt, s.Nd), dtype=torch.float64, device=dev)
    mout = torch.empty((s.Nt, s.Nm), dtype=torch.float64, device=dev)

    def step():
        op.matvec(mt, out=dout)
        op.rmatvec(dt, out=mout)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    ms_per_step = elapsed / args.steps * 1e3
    value = 2 * args.steps / elapsed
    log(f"fp64 step {ms_per_step:.3f} ms -> {value:.1f} matvecs/s")

    # per-kernel durations from HIP events on the launch stream (separate pass)
    op.profile(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = op.profile_read()
    op.profile(False)
    kms = {"fwd": prof["fwd"], "adj": prof["adj"]}
    fwd_ms, adj_ms = sum(prof["fwd"]), sum(prof["adj"])
    gb_fwd = gemv_bytes(s, 16) / (prof["fwd"][1] * 1e-3) / 1e9
    gb_adj = gemv_bytes(s, 16) / (prof["adj"][1] * 1e-3) / 1e9
    log(f"kernels fwd {['%.4f' % x for x in prof['fwd']]} adj {['%.4f' % x for x in prof['adj']]} ms; "
        f"product {gb_fwd:.0f} / {gb_adj:.0f} GB/s")
    got_d, got_m = dout.cpu().numpy(), mout.cpu().numpy()

    # CPU oracle: timed baseline and reference for the errors
    import oracle
    if args.no_oracle:
        ref_d, ref_m = got_d, got_m
    t2 = time.perf_counter()
    if not args.no_oracle:
        ref_d = oracle.forward(F, m)
    t3 = time.perf_counter()
    if not args.no_oracle:
        ref_m = oracle.adjoint(F, d)
    t4 = time.perf_counter()
    try:
        from threadpoolctl import threadpool_info
        cores = max((i.get("num_threads") or 1) for i in threadpool_info()) if threadpool_info() else 1
    except Exception:
        cores = os.cpu_count()
    cpu_baseline = None
    if not args.no_cpu_baseline:
        cpu_model = None
        try:
            with open("/proc/cpuinfo") as fh:
                cpu_model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), None)
        except OSError:
            pass
        cpu_baseline = {"value": 2.0 / (t4 - t2), "unit": "matvecs/s", "cores": int(cores), "kind": "oracle",
                        "cpu_model": cpu_model, "host_cpus": os.cpu_count(),
                        "sample": f"one forward ({t3 - t2:.2f}s) and one adjoint ({t4 - t3:.2f}s) float64 "
                                  "oracle matvec at Nt=1000, Nd=100, Nm=5000, whole vectors"}
        try:
            from threadpoolctl import threadpool_limits
            with threadpool_limits(limits=1):
                t5 = time.perf_counter()
                oracle.forward(F, m)
                t6 = time.perf_counter()
            cpu_baseline["single_thread"] = {"value": 1.0 / (t6 - t5), "unit": "matvecs/s", "cores": 1,
                                             "sample": f"one forward float64 oracle matvec at the same shape, "
                                                       f"one thread ({t6 - t5:.2f}s)"}
            log(f"cpu oracle, one thread: forward {t6 - t5:.2f}s")
        except Exception as exc:  # threadpoolctl missing: report without the one-thread figure
            log(f"no one-thread oracle timing: {exc}")
    rel = None if args.no_oracle else {"fwd": oracle.relative_l2(got_d, ref_d),
                                       "adj": oracle.relative_l2(got_m, ref_m)}
    if rel:
        log(f"fp64 rel err fwd {rel['fwd']:.3e} adj {rel['adj']:.3e}; oracle {t4 - t2:.1f}s")

    mixed = None
    if args.mixed != "none":
        confs = all_configs() if args.mixed == "all" else ds_configs() + HALF_CONFIGS
        mixed = mixed_section(log, op, s, mt, dt, dout, mout, ref_d, ref_m, confs)

    paper_multi = None
    if not args.no_multi_rhs and not args.multi_rhs_products_only:
        # many right-hand sides and the data-space Hessian at the paper's shape
        g = torch.Generator(device=dev)
        g.manual_seed(2508_10202 + 100 * 2 + 3)
        M64 = torch.randn((64, s.Nt, s.Nm), dtype=torch.float64, device=dev, generator=g)
        D64 = torch.randn((64, s.Nt, s.Nd), dtype=torch.float64, device=dev, generator=g)
        paper_multi = {"nrhs_sweep": {prec: nrhs_sweep(op, s, M64, D64, prec) for prec in ("ddsdd", "ddddd")}}
        log("paper-shape nrhs sweep: " + json.dumps(paper_multi["nrhs_sweep"]))
        del M64, D64
        paper_multi["hessian"] = hessian_section(log, op, F, s, "Nt=1000 Nd=100 Nm=5000")
        op.set_precision(fwd="ddddd", adj="ddddd")
    multi = None if args.no_multi_rhs else multi_rhs_section(log, args.multi_rhs_products_only)
    sbg = None if args.no_multi_rhs or args.multi_rhs_products_only else sbgemv_section(log)
    serving = None
    if args.serving_seconds > 0:
        op.close()
        serving = serving_section(log, args.serving_seconds, budget_gib=args.serving_budget_gib)

    achieved = gb_fwd
    roofline = {"bound": "hbm", "kernel": "gemv_fwd_kernel<s_f64,double,double,double> (phase 3, float64)",
                "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic_record(),
                "algorithmic_bytes_per_launch": gemv_bytes(s, 16), "avg_launch_ms": round(prof["fwd"][1], 5),
                "adjoint": {"kernel": "gemv_adj_kernel<s_f64,double,double,double>", "achieved": round(gb_adj, 1),
                            "frac": round(gb_adj / PEAK_HBM_GBS, 4), "avg_launch_ms": round(prof["adj"][1], 5)}}
    rec = {
        "metric": METRIC, "value": round(value, 2), "unit": "matvecs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "fftmatvec forward + adjoint, float64, Nt=1000 Nd=100 Nm=5000, L=2000, 1 vector",
                   "Nt": s.Nt, "Nd": s.Nd, "Nm": s.Nm, "nrhs": 1, "parallelism": "single-gpu"},
        "hbm_gbs": {"fwd": round(matvec_bytes(s, 16) / (fwd_ms * 1e-3) / 1e9, 1),
                    "adj": round(matvec_bytes(s, 16) / (adj_ms * 1e-3) / 1e9, 1)},
        "kernels_ms": kms, "rel_err": rel, "roofline": roofline, "cpu_baseline": cpu_baseline,
        "mixed": mixed, "multi_rhs": multi, "paper_shape_multi_rhs": paper_multi, "serving": serving,
        "sbgemv": sbg,
    }
    op.close()
    if args.copy_calibration_gib > 0:
        n = int(args.copy_calibration_gib * 2 ** 30) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        rec["copy_calibration_bytes"] = n * 8
        log(f"copy calibration: 3 x {n * 8} bytes")
    if args.json_out:
        with open(args.json_out, "w") as fh:
            json.dump(rec, fh, indent=1)
    short = dict(rec)
    if mixed:
        short["mixed"] = {"n_configs": mixed["n_configs"], "best": mixed["best"], "pareto": mixed["pareto"],
                          "out_of_window": mixed["out_of_window"], "ds_subset": mixed["ds_subset"]}
    if sbg:
        short["sbgemv"] = {f'{r["type"]}{r["op"]} m={r["m"]}': {"gbs": r["gbs"], "frac": r["frac"]} for r in sbg}
    print(json.dumps(short), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
