"""Benchmark: FP64 eigensolves/s of the preconditioned Jacobi pipeline at n = 2048.

One step = one preconditioned solve (FP32 eigensolve -> FP64 MGS -> FP64 Q^T A Q -> FP64
round-robin Jacobi sweeps) of each of three n = 2048 matrices A = Q diag(lambda) Q^T (Haar Q)
with lambda ~ U[-1,1], a signed geometric spectrum 10^(-8 i/(n-1)), and ten clusters of width
1e-6.  Inputs are resident in device memory before the timed region.  Printed beside it: plain
FP64 Jacobi on the same matrices, sweep counts, residuals, the dominant kernel's roofline figure
(HIP events around each run of one class's launches, in one more untimed pass), the learned start
at n = 256 (the size where the network is feasible), the batched path on 4096 matrices of sizes
32..512 next to a per-matrix loop, and the CPU oracle timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 2048] [--variant auto]
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

METRIC = "FP64 eigensolves/sec + Jacobi sweeps at n=2048: precond & MLP vs plain, resid<=1e-13"
HBM_PEAK_GBS = 8000.0
PEAK = {"fp64_mfma": 78.6, "fp32_mfma": 157.3, "fp64_valu": 78.6, "fp32_valu": 157.3}   # TFLOP/s
TILE = 64   # 2b: block-pair size of the blocked variant


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def elem_bytes(n: int, dtype_bytes: int, steps: int, rotations: int) -> float:
    """Algorithmic bytes of `steps` element-wise steps that applied `rotations` rotations: T is
    read and written in full every step; V moves only the two columns of an applied rotation
    (read and written: 4 n entries)."""
    return dtype_bytes * (steps * n * (n + 1) + rotations * 4 * n)


KERNEL_OF = {"tridiag_reduce": ("sytrd_reg_kernel",),
             "tridiag_rest": ("tri_bisect_kernel", "tri_vectors_kernel", "bt_tfactor_kernel"),
             "inner64": ("blk_inner_kernel<double", "blk_inner_v_kernel<double"),
             "update64": ("blk_update16_kernel<double",),
             "inner32": ("blk_inner_kernel<float", "blk_inner_v_kernel<float"),
             "update32": ("blk_update16_kernel<float",),
             "elem64": ("elem_step_kernel<double",), "elem32": ("elem_step_kernel<float",)}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_n2048.json")
# the source file that holds each class's kernels (its digest at counter time gates the figure)
SOURCE_OF = {"tridiag_reduce": "tridiag.hip", "tridiag_rest": "tridiag.hip", "inner64": "blocked.hip",
             "update64": "blocked.hip", "inner32": "blocked.hip", "update32": "blocked.hip",
             "elem64": "elem.hip", "elem32": "elem.hip"}


def measured_traffic(cls: str):
    """HBM bytes per launch of a kernel class from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary (copy-kernel scaled), or None when there is none or the source file that holds the
    class's kernels changed since the counters were taken."""
    import hashlib
    try:
        t = json.load(open(TRAFFIC_FILE))
        gated = [src for src in t["sources"] if os.path.basename(src) == SOURCE_OF.get(cls)]
        if not gated:
            return None
        for src in gated:
            if hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest() != t["sources"][src]:
                return None
        sel = [v for k, v in t["kernels"].items() if any(p in k for p in KERNEL_OF.get(cls, ()))]
        calls = sum(v["dispatches"] for v in sel)
        if not calls:
            return None
        return sum(v["bytes"] * v["dispatches"] for v in sel) / calls
    except (OSError, KeyError, ValueError):
        return None


def roofline_for(cls: str, k: dict, n: int, rotations: int) -> dict:
    """Roofline figure of one kernel class from its HIP-event launch times (runs of launches).
    update*: algorithmic flops of the block rotations actually applied: each (2b)x(2b) tile
    W_k^T T W_l costs 2 * 2(2b)^3, each 2b-row chunk of V W_k costs 2(2b)^3.
    elem*: algorithmic bytes of the steps (elem_bytes: T in full, V for the applied rotations).
    inner*: rotation flops (each rotation of a 2b x 2b subproblem updates two rows and two
    columns of S and two columns of E: about 12 * 2b flops) on the vector units, plus the V
    chunks (2 (2b)^3 flop each) the same launches update for the previous block step."""
    ms, launches = k["ms"], max(k["launches"], 1)
    avg_s = ms / 1e3 / launches
    if cls == "tridiag_reduce":
        # Householder tridiagonalization: (4/3) n^3 flops (symmetric rank-2 updates and products
        # with the trailing matrix), FP32 operands; bound in practice by the n - 2 sequential
        # column exchanges between the workgroups, placed against the FP32 vector peak
        flops = 4.0 / 3.0 * n ** 3
        ach = flops / avg_s / 1e12
        return {"bound": "alu", "achieved": round(ach, 4), "peak": PEAK["fp32_valu"], "unit": "TFLOP/s",
                "frac": round(ach / PEAK["fp32_valu"], 6), "traffic": measured_traffic(cls), "kernel": "sytrd_reg_kernel",
                "avg_launch_us": round(avg_s * 1e6, 3), "algorithmic_flops_per_launch": flops,
                "launches_timed": k["launches"], "per_column_us": round(avg_s * 1e6 / max(n - 2, 1), 3)}
    if cls == "tridiag_rest":
        # bisection and eigenvectors of T (O(n^2) each) and the back-transformation Z = Q Y, 2 n^3
        # flops on the FP64 matrix cores
        flops = 2.0 * n ** 3
        ach = flops / avg_s / 1e12
        return {"bound": "mfma", "achieved": round(ach, 4), "peak": PEAK["fp64_mfma"], "unit": "TFLOP/s",
                "frac": round(ach / PEAK["fp64_mfma"], 6), "traffic": None,
                "kernel": "tri_bisect_kernel + tri_vectors_kernel + back-transformation GEMMs",
                "avg_launch_us": round(avg_s * 1e6, 3), "algorithmic_flops_per_launch": flops,
                "launches_timed": k["launches"]}
    if cls.startswith("update"):
        flops = k["tiles"] * 4 * TILE ** 3 + k["chunks"] * 2 * TILE ** 3
        per_launch = flops / launches
        peak = PEAK["fp64_mfma" if cls.endswith("64") else "fp32_mfma"]
        ach = per_launch / avg_s / 1e12
        return {"bound": "mfma", "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(ach / peak, 4), "traffic": measured_traffic(cls), "kernel": ">, ".join(KERNEL_OF[cls]) + ">",
                "avg_launch_us": round(avg_s * 1e6, 3), "algorithmic_flops_per_launch": per_launch,
                "launches_timed": k["launches"]}
    if cls.startswith("elem"):
        db = 8 if cls.endswith("64") else 4
        bpl = elem_bytes(n, db, launches, rotations) / launches
        ach = bpl / avg_s / 1e9
        return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(cls), "kernel": f"elem_step_kernel<{cls[-2:]}>",
                "avg_launch_us": round(avg_s * 1e6, 3), "algorithmic_bytes_per_launch": bpl,
                "launches_timed": k["launches"]}
    # inner launches after a sweep's first block step also carry the whole update of the previous
    # step on the matrix cores: its V chunks (2 (2b)^3 flop each) and T tiles (4 (2b)^3 each,
    # counted once also where two inner workgroups compute the same tile); those dominate the
    # launch's flops, so the launch is placed on the matrix-core roofline
    rot_flops = rotations * 12 * TILE
    v_flops = k.get("chunks", 0) * 2 * TILE ** 3 + k.get("tiles", 0) * 4 * TILE ** 3
    per_launch = (rot_flops + v_flops) / launches
    bound = "mfma" if v_flops > rot_flops else "alu"
    peak = PEAK[("fp64_" if cls.endswith("64") else "fp32_") + ("mfma" if bound == "mfma" else "valu")]
    ach = per_launch / avg_s / 1e12
    return {"bound": bound, "achieved": round(ach, 4), "peak": peak, "unit": "TFLOP/s",
            "frac": round(ach / peak, 6), "traffic": measured_traffic(cls),
            "kernel": f"blk_inner_v_kernel<{cls[-2:]}> (+ blk_inner_kernel at step 0)",
            "avg_launch_us": round(avg_s * 1e6, 3), "algorithmic_flops_per_launch": per_launch,
            "rotation_flops_per_launch": rot_flops / launches, "update_flops_per_launch": v_flops / launches,
            "launches_timed": k["launches"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--variant", default="auto")
    ap.add_argument("--tol", type=float, default=0.0, help="<= 0: the paper's 20 * 2^-53")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-n", type=int, default=1024, help="order of the CPU oracle's full solve")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-Jacobi comparison")
    ap.add_argument("--no-mlp", action="store_true", help="skip the learned-start row at n=256")
    ap.add_argument("--no-elem", action="store_true", help="skip the element-wise variant's step rooflines")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-path row (4096 matrices)")
    ap.add_argument("--no-ex62", action="store_true", help="skip the multiple-eigenvalue study rows")
    ap.add_argument("--no-prec", action="store_true", help="skip the FP16 / BF16 step-1 study")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched-path row and print it (for profiling that path)")
    ap.add_argument("--batched-noloop", action="store_true",
                    help="batched row without its per-matrix comparison loop")
    ap.add_argument("--mlp-train", type=int, default=4096, help="training solves for the learned-start row")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        nb = args.copy_probe << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nb, "copies": 5}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2211_03339_amd import jacobi
    from paper_2211_03339_amd import testmats as tm

    jacobi.load()
    if args.batched_only:
        print(json.dumps({"batched_4096": batched_row(loop_sample=0 if args.batched_noloop else 128)}), flush=True)
        return
    n = args.n
    spectra = list(tm.SPECTRA)
    log(f"[bench] generating {len(spectra)} matrices of order {n}")
    mats = [tm.precond_case(n, k) for k in spectra]
    dev = [torch.from_numpy(A).cuda() for A, _ in mats]   # symmetric: row/column-major agree
    Ws = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in mats]
    Vs = [torch.empty((n, n), dtype=torch.float64, device="cuda") for _ in mats]
    stream = torch.cuda.current_stream()
    sp = jacobi.ctypes.c_void_p(stream.cuda_stream)

    def solve(i, precond, stats, profile=0):
        o = jacobi._opts(precond, args.variant, profile=profile)
        code = jacobi.syev_jacobi_raw(dev[i].data_ptr(), n, n, Ws[i].data_ptr(), Vs[i].data_ptr(), n,
                                      args.tol, o, stats, sp)
        if code != 0:
            raise RuntimeError(f"syev_jacobi_ex returned {code}: {jacobi.last_error()}")

    stats = [jacobi.JacStats() for _ in mats]
    for w in range(args.warmup):
        for i in range(len(mats)):
            solve(i, "fp32", stats[i])
        log(f"[bench] warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_s = []
    for k in range(args.steps):
        ts = time.perf_counter()
        for i in range(len(mats)):
            solve(i, "fp32", stats[i])   # synchronous: returns after the solve has completed
        step_s.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"[bench] timed {args.steps} steps in {elapsed:.3f} s")
    # Per-kernel-class launch times come from one more, untimed pass with HIP events around each run
    # of consecutive launches of one class (a sweep's inner launches, its final update, an element
    # sweep's steps), divided by the run's launch count; the events stay out of the timed region.
    kern = {}
    rot = {"64": 0, "32": 0}
    prof_ms = 0.0
    for i in range(len(mats)):
        pst = jacobi.JacStats()
        solve(i, "fp32", pst, profile=1)
        d = pst.as_dict()
        prof_ms += d["stage_ms"]["total"]
        rot["64"] += d["rotations"]
        rot["32"] += d["fp32_rotations"]
        for name, kv in d["kernels"].items():
            a = kern.setdefault(name, {"ms": 0.0, "launches": 0, "tiles": 0, "chunks": 0})
            for f in a:
                a[f] += kv[f]
    torch.cuda.synchronize()
    solves = args.steps * len(mats)
    value = solves / elapsed

    per_spec = {}
    for i, (A, lam) in enumerate(mats):
        W = Ws[i].cpu().numpy()
        V = Vs[i].t().cpu().numpy()
        res = float(np.linalg.norm(A @ V - V * W[None, :]) / np.linalg.norm(A))
        orth = float(np.linalg.norm(V.T @ V - np.eye(n)))
        lam_err = float(np.abs(W - np.sort(lam)).max() / np.abs(lam).max())
        st = stats[i].as_dict()
        per_spec[spectra[i]] = {"sweeps": st["sweeps"], "fp32_sweeps": st["fp32_sweeps"],
                                "stage1": {0: "none", 1: "fp32 jacobi", 2: "fp32 tridiagonal"}[st["fp32_method"]],
                                "JU": round(st["rotations"] / (n * (n - 1) / 2), 3),
                                "res": res, "orth": orth, "orth_over_sqrt_n": orth / np.sqrt(n),
                                "lam_err_rel": lam_err,
                                "stage_ms": {k2: round(v, 3) for k2, v in st["stage_ms"].items()}}
    log(f"[bench] accuracy checked: {json.dumps({k: (v['res'], v['sweeps']) for k, v in per_spec.items()})}")

    plain = None
    if not args.no_plain:
        # plain FP64 Jacobi on the same matrices, with the same warm-up and step counts
        pst = [jacobi.JacStats() for _ in mats]
        for w in range(args.warmup):
            for i in range(len(mats)):
                solve(i, "none", pst[i])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pstep_s = []
        for k in range(args.steps):
            ts = time.perf_counter()
            for i in range(len(mats)):
                solve(i, "none", pst[i])
            pstep_s.append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        pt = time.perf_counter() - t1
        med_pre, med_plain = float(np.median(step_s)), float(np.median(pstep_s))
        plain = {"solves_per_s": len(mats) * args.steps / pt,
                 "sweeps": {spectra[i]: pst[i].sweeps for i in range(len(mats))},
                 "ms_per_step": {"median": round(med_plain * 1e3, 3), "min": round(min(pstep_s) * 1e3, 3),
                                 "max": round(max(pstep_s) * 1e3, 3)},
                 "speedup_precond_vs_plain": round(value / (len(mats) * args.steps / pt), 4),
                 "speedup_spread": {"median_step": round(med_plain / med_pre, 4),
                                    "worst_step": round(min(pstep_s) / max(step_s), 4),
                                    "best_step": round(max(pstep_s) / min(step_s), 4)}}
        log(f"[bench] plain: {plain}")

    # Step 1 at lower precision (FP16, BF16: A and the step-1 eigenvectors rounded to it), the
    # paper's precision study: start quality, FP64 sweeps and solve time per spectrum (one warm
    # and one measured solve each, outside the timed region).
    prec_study = None
    if not args.no_prec:
        prec_study = {}
        for prec in ("fp16", "bf16"):
            row = {}
            for i in range(len(mats)):
                o = jacobi._opts("fp32", args.variant, stage1_prec=prec)
                pstat = jacobi.JacStats()
                for _ in range(2):
                    code = jacobi.syev_jacobi_raw(dev[i].data_ptr(), n, n, Ws[i].data_ptr(), Vs[i].data_ptr(), n,
                                                  args.tol, o, pstat, sp)
                    if code != 0:
                        raise RuntimeError(f"syev_jacobi_ex ({prec} step 1) returned {code}: {jacobi.last_error()}")
                torch.cuda.synchronize()
                d = pstat.as_dict()
                A, lam = mats[i]
                W = Ws[i].cpu().numpy()
                row[spectra[i]] = {"off0_rel": d["off0"] / d["nrmA"], "sweeps": d["sweeps"],
                                   "ms_total": round(d["stage_ms"]["total"], 3),
                                   "lam_err_rel": float(np.abs(W - np.sort(lam)).max() / np.abs(lam).max())}
            prec_study[prec] = row
        prec_study["fp32"] = {spectra[i]: {"off0_rel": stats[i].off0 / stats[i].nrmA, "sweeps": stats[i].sweeps,
                                           "ms_total": round(float(stats[i].stage_ms[5]), 3)}
                              for i in range(len(mats))}
        log(f"[bench] precision study: {json.dumps(prec_study)}")

    # Roofline of the dominant kernel (by measured launch time inside the timed region).
    dom = max(kern, key=lambda c: kern[c]["ms"])
    roofline = roofline_for(dom, kern[dom], n, rot.get(dom[-2:], 0))
    kernels = {c: {"ms_total": round(v["ms"], 3), "launches": v["launches"],
                   "share_of_profiled_step": round(v["ms"] / prof_ms, 4)} for c, v in kern.items()}
    others = {c: roofline_for(c, kern[c], n, rot.get(c[-2:], 0)) for c in kern if c != dom}

    # The element-wise variant (n/2 disjoint rotations per launch, T and V streamed through HBM):
    # one profiled preconditioned solve of the U[-1,1] matrix, for its step kernels' rooflines.
    elem = None
    if not args.no_elem:
        est = jacobi.JacStats()
        o = jacobi._opts("fp32", "element", profile=1)
        code = jacobi.syev_jacobi_raw(dev[0].data_ptr(), n, n, Ws[0].data_ptr(), Vs[0].data_ptr(), n, args.tol, o,
                                      est, sp)
        if code != 0:
            raise RuntimeError(f"syev_jacobi_ex (element) returned {code}: {jacobi.last_error()}")
        torch.cuda.synchronize()
        ed = est.as_dict()
        elem = {"ms_total": round(ed["stage_ms"]["total"], 3), "sweeps": ed["sweeps"], "fp32_sweeps": ed["fp32_sweeps"],
                "rooflines": {c: roofline_for(c, v, n, ed["rotations"] if c == "elem64" else ed["fp32_rotations"])
                              for c, v in ed["kernels"].items() if c.startswith("elem")}}
        log(f"[bench] element variant: {json.dumps(elem)}")

    ex62 = None
    if not args.no_ex62:
        ex62 = example62_rows(n)
        log(f"[bench] multiple eigenvalues (Example 6.2 recipe): {json.dumps(ex62)}")

    bat_row = None
    if not args.no_batched:
        bat_row = batched_row()
        log(f"[bench] batched path: {json.dumps(bat_row)}")

    mlp_row = None
    if not args.no_mlp:
        mlp_row = learned_row(args.mlp_train)
        log(f"[bench] learned start n=256: {json.dumps(mlp_row)}")

    cpu = None
    if not args.no_cpu:
        import oracle
        ns = args.cpu_n
        A, lam = tm.precond_case(ns, "uniform")
        log(f"[bench] CPU oracle: one full plain-Jacobi solve, n={ns}")
        tc = time.perf_counter()
        r = oracle.syev(A, tol=args.tol if args.tol > 0 else oracle.DEFAULT_TOL)
        dt = time.perf_counter() - tc
        cpu = {"value": round(1.0 / dt, 6), "unit": "eigensolves/s", "cores": 1, "kind": "oracle", "n": ns,
               "sample": f"one full oracle solve (row-cyclic Jacobi, FP64, 1 thread) of the {ns}x{ns} "
                         f"U[-1,1] matrix of the same family: {dt:.2f} s, {r.sweeps} sweeps (measured at "
                         f"n={ns}, not scaled to n={n})",
               "cpu": _cpu_model()}

    out = {"metric": METRIC, "value": round(value, 4), "unit": "eigensolves/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 3),
           "ms_per_step_spread": {"median": round(float(np.median(step_s)) * 1e3, 3),
                                  "min": round(min(step_s) * 1e3, 3), "max": round(max(step_s) * 1e3, 3)},
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"preconditioned pipeline (FP32 eig -> FP64 MGS -> FP64 Q^T A Q -> "
                                  f"FP64 round-robin Jacobi), n={n}, spectra U[-1,1] / signed geometric "
                                  f"1e-8 / 10 clusters x 1e-6, one solve of each per step",
                      "n": n, "solves_per_step": len(mats), "variant": args.variant,
                      "tol": args.tol if args.tol > 0 else 20 * 2.0 ** -53},
           "per_spectrum": per_spec, "plain": plain, "learned_n256": mlp_row, "batched_4096": bat_row, "element_variant": elem,
           "example62_study": ex62, "precision_study": prec_study,
           "roofline": roofline,
           "cpu_baseline": cpu,
           "kernels": kernels, "other_rooflines": others}
    print(json.dumps(out), flush=True)


def learned_row(n_train: int, n_eval: int = 32, epochs: int = 8):
    """Learned start on the n = 256 family (the network row of the metric at the size where it is
    feasible), as the trainer runs it: the network starts as the constant start Z0 (eigenvectors of
    A0), its targets are n_train method-generated solves aligned to Z0 within windows of nearby
    eigenvalues, and the
    parameters with the best start residual on 16 validation matrices are kept; then solves of
    held-out matrices with the learned start (FP32 fallback), the constant start, the FP32 start and
    plain Jacobi are timed."""
    from paper_2211_03339_amd import learned
    from paper_2211_03339_amd import testmats as tm
    n = 256
    A0, B = learned.family(n)
    Z0, lam0 = learned.constant_start(A0, with_eigenvalues=True)
    theta, T, data = learned.make_dataset(A0, B, tm.param_thetas(n_train, learned.THETA_TRAIN_SEED), Z0=Z0,
                                          lam0=lam0)
    net = learned.jacobi.Mlp(8, 1024, n, 256, seed=0)
    learned.init_as_correction(net, Z0)
    val = learned.validation_set(A0, B, tm.param_thetas(16, learned.THETA_VAL_SEED))
    tr = learned.train(net, theta, T, epochs=epochs, batch=256, lr=1e-4, weight_decay=0.0, val=val)
    del T
    ev = learned.evaluate(net, A0, B, tm.param_thetas(n_eval, learned.THETA_EVAL_SEED), check=True, Z0=Z0)
    net.close()
    modes = ("mlp", "const", "fp32", "plain", "mlp_forced")
    return {"n": n, "train_solves": n_train, "epochs": epochs, "data_s": round(data["seconds"], 3),
            "train_s": round(tr["seconds"], 3), "final_loss": tr["loss_per_epoch"][-1],
            "val_start_resid": [round(x, 4) for x in tr["val_start_resid"]], "kept_epoch": tr["kept_epoch"],
            "eval_matrices": n_eval,
            "solves_per_s": {m: round(1e3 / ev[m]["mean_ms"], 2) for m in modes},
            "mean_sweeps": {m: ev[m]["mean_sweeps"] for m in modes},
            "max_res": max(ev[m]["max_res"] for m in modes),
            "learned_start": ev["learned_start"], "const_start": ev["const_start"]}


def example62_rows(n: int, kappas=(1e3, 1e6), r: int = 4):
    """Multiple eigenvalues (Example 6.2, the shapes of its result tables): A = P diag(lam kron 1_r)
    P^T with r = 4, P Haar (the library's MGS of a seeded Gaussian on the device) and lam by mode 1-5 and kappa,
    solved preconditioned and plain.  Per case: ||off(Q^T A Q)||_F of the start, d(A)/4 (a quarter
    of the smallest gap between distinct eigenvalues), the residual ||A V - V W||_F / ||A||_F,
    ||V^T V - I||_F (raw and / sqrt(n)), the start and sweep times and the FP64 sweeps."""
    import torch
    from paper_2211_03339_amd import jacobi
    from paper_2211_03339_amd import testmats as tm
    s = n // r
    rows = []
    gen = torch.Generator(device="cuda")
    for kappa in kappas:
        for mode in range(1, 6):
            g = tm.rng(6200 + mode)
            if mode == 1:
                lam = np.full(s, 1.0 / kappa); lam[0] = 1.0
            elif mode == 2:
                lam = np.ones(s); lam[-1] = 1.0 / kappa
            elif mode == 3:
                lam = kappa ** np.linspace(-1.0, 0.0, s)
            elif mode == 4:
                lam = 1.0 - (1.0 - 1.0 / kappa) * np.linspace(0.0, 1.0, s)
            else:
                lam = kappa ** (-g.uniform(size=s))
            full = torch.from_numpy(np.kron(lam, np.ones(r))).cuda()
            gen.manual_seed(620_000 + mode)
            Q = jacobi.jac_mgs(torch.randn((n, n), dtype=torch.float64, device="cuda", generator=gen)).contiguous()
            A = (Q * full.unsqueeze(0)) @ Q.t().contiguous()
            A = (0.5 * (A + A.t())).contiguous()
            u = np.unique(lam)
            dA = float(np.min(np.diff(u))) / 4 if u.size > 1 else float("inf")
            row = {"mode": mode, "kappa": kappa, "d_over_4": dA}
            nA = float(torch.linalg.norm(A))
            eye = torch.eye(n, dtype=torch.float64, device="cuda")
            for pre in ("fp32", "none"):
                jacobi.syev_jacobi_ex(A, precond=pre)   # warm
                torch.cuda.synchronize()
                W, V, st, _ = jacobi.syev_jacobi_ex(A, precond=pre)
                torch.cuda.synchronize()
                Vc = V.contiguous()
                res = float(torch.linalg.norm(A @ Vc - Vc * W.unsqueeze(0))) / nA
                orth = float(torch.linalg.norm(Vc.t().contiguous() @ Vc - eye))
                lam_err = float((W - torch.sort(full).values).abs().max())
                ms = st["stage_ms"]
                row[pre] = {"sweeps": st["sweeps"], "res": res, "orth": orth, "orth_over_sqrt_n": orth / n ** 0.5,
                            "lam_err": lam_err, "ms_total": round(ms["total"], 2),
                            "ms_start": round(ms["start"] + ms["mgs"] + ms["similarity"], 2),
                            "ms_sweeps": round(ms["sweeps"], 2)}
                if pre == "fp32":
                    row["off_QtAQ"] = st["off0"]
            rows.append(row)
            del A, Q
    return {"n": n, "r": r, "cases": rows,
            "total_ms_precond": round(sum(c["fp32"]["ms_total"] for c in rows), 1),
            "total_ms_plain": round(sum(c["none"]["ms_total"] for c in rows), 1)}


def batched_row(count: int = 4096, loop_sample: int = 128, reps: int = 3):
    """The batched path on its own workload: `count` matrices A = Q diag(lambda) Q^T with sizes
    32 * U{1..16} (seed 3), Haar Q, lambda ~ U[-1,1], plain and preconditioned (Algorithm 4.1 per
    matrix).  Each form: the autotuner, a capturing first call, then `reps` timed calls (graph
    replay plus the convergence check); next to it a per-matrix loop through the single-matrix
    call on the first `loop_sample` matrices.  The inputs are built on the device (seeded Gaussian
    matrices orthonormalised by the library's MGS) so that the bench does not spend minutes in host
    QRs.
    Roofline: FP64 matrix-core work of the blocked sweeps, 12 n^3 flop per FP64 sweep of an order-n
    matrix (T updated as 8 n^3, V as 4 n^3), over the wall time of a call, against the FP64 peak."""
    import torch
    from paper_2211_03339_amd import jacobi
    from paper_2211_03339_amd import testmats as tm
    sizes = [int(x) for x in tm.batched_sizes(count, 3)]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3_000_003)
    mats = [None] * count
    lams = [None] * count
    for nval in sorted(set(sizes)):
        idx = [i for i, x in enumerate(sizes) if x == nval]
        G = torch.randn((len(idx), nval, nval), dtype=torch.float64, device="cuda", generator=gen)
        # Haar factors: the orthonormal QR factor (positive R diagonal) of each Gaussian matrix,
        # by the library's MGS
        Q = torch.stack([jacobi.jac_mgs(G[j]).contiguous() for j in range(len(idx))])
        lam = torch.rand((len(idx), nval), dtype=torch.float64, device="cuda", generator=gen) * 2 - 1
        A = torch.matmul(Q * lam.unsqueeze(-2), Q.transpose(-2, -1).contiguous())
        A = 0.5 * (A + A.transpose(-2, -1).contiguous())
        for j, i in enumerate(idx):
            mats[i] = A[j].contiguous()
            lams[i] = lam[j]
        del G, Q, A
    torch.cuda.synchronize()
    b = jacobi.Batch(mats)
    ns = min(loop_sample, count)
    cube = sum(x ** 3 for x in sizes)
    cube_s = max(sum(x ** 3 for x in sizes[:ns]), 1)
    row = {"matrices": count, "sizes": "32*U{1..16}, seed 3", "mean_n": round(sum(sizes) / count, 1)}
    for pre in ("none", "fp32"):
        t0 = time.perf_counter()
        b.autotune(precond=pre)
        torch.cuda.synchronize()
        tune_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        b.run(precond=pre)
        torch.cuda.synchronize()
        first_s = time.perf_counter() - t0
        per = []
        for _ in range(reps):
            t0 = time.perf_counter()
            b.run(precond=pre)
            torch.cuda.synchronize()
            per.append(time.perf_counter() - t0)
        run_s = float(np.median(per))
        W, V, sw, info = b.results()
        s32 = b.sweeps32.cpu().numpy()
        # accuracy on every 16th matrix, against its known spectrum and by the defining properties
        worst = {"res": 0.0, "orth": 0.0, "lam_err": 0.0}
        for i in range(0, count, 16):
            A, w, v = mats[i], W[i], V[i].contiguous()
            nA = float(torch.linalg.norm(A))
            worst["res"] = max(worst["res"], float(torch.linalg.norm(A @ v - v * w[None, :])) / nA)
            eye = torch.eye(A.shape[0], dtype=torch.float64, device="cuda")
            worst["orth"] = max(worst["orth"], float(torch.linalg.norm(v.t().contiguous() @ v - eye)))
            lam_sorted = torch.sort(lams[i]).values
            worst["lam_err"] = max(worst["lam_err"], float((w - lam_sorted).abs().max() / lam_sorted.abs().max()))
        # the per-matrix loop through the single-matrix call on a sample
        loop_s = loop_proj = float("nan")
        if ns:
            for i in range(2):
                jacobi.syev_jacobi_ex(mats[i], precond=pre)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(ns):
                jacobi.syev_jacobi_ex(mats[i], precond=pre)
            torch.cuda.synchronize()
            loop_s = time.perf_counter() - t0
            loop_proj = loop_s * cube / cube_s
        flops64 = float(sum(12.0 * n ** 3 * int(k) for n, k in zip(sizes, sw)))
        achieved = flops64 / run_s / 1e12
        row[pre] = {"autotune_s": round(tune_s, 3), "first_call_s": round(first_s, 3), "call_s": round(run_s, 4),
                    "call_s_spread": [round(x, 4) for x in per],
                    "matrices_per_s": round(count / run_s, 1), "unconverged": int((info != 0).sum()),
                    "mean_sweeps": round(float(sw.mean()), 2), "max_sweeps": int(sw.max()),
                    "mean_fp32_sweeps": round(float(s32.mean()), 2), "stats": b.stats,
                    "tuned_n512": jacobi.jac_tune_entry(512, pre),
                    "loop_sample": ns, "loop_sample_s": round(loop_s, 4) if ns else None,
                    "loop_projected_s": round(loop_proj, 3) if ns else None,
                    "speedup_vs_loop": round(loop_proj / run_s, 2) if ns else None,
                    "roofline_fp64_sweeps": {"bound": "mfma", "achieved": round(achieved, 3), "peak": 78.6,
                                             "unit": "TFLOP/s", "frac": round(achieved / 78.6, 4),
                                             "work": "12 n^3 per FP64 sweep, summed over the batch"},
                    "checked_every_16th": {k: float("%.3g" % v) for k, v in worst.items()}}
        log(f"[bench] batched {pre}: {json.dumps(row[pre])}")
    row["speedup_precond_vs_plain"] = round(row["none"]["call_s"] / row["fp32"]["call_s"], 3)
    return row


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip() + f" ({os.cpu_count()} logical CPUs)"
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
