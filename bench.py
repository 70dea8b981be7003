#!/usr/bin/env python3
"""Throughput of the randomized orthogonal projection on one MI355X.

One step = the whole path on one batch of work: precondition A (sketch,
pivoted QR, R^{-T}, P^{-1}A, Gram, its inverse) and project k right-hand sides
(least-squares x, row projection A^T x, null projection b - A^T x, with the
compensated refinement), all through the C ABI.

Workloads (seeded synthetic inputs, A = U diag(sigma) V^T with Haar factors):
  mixed_2048x262144 (default) m=2048, n=262144, sigma 1 -> 1e-8, l=8192, k=64;
                             the split-bfloat16 Gram form (main line)
                             against the binary32-Gram, binary64 and
                             bfloat16 forms on the same inputs
  plain_512x65536            m=512, n=65536, sigma 1 -> 1e-10, l=2048, k=16;
                             binary64, plus the mixed forms on the same inputs
  plain_64x4096              m=64, n=4096, sigma 1 -> 1e-6, l=256, k=1
  batch_256                  256 members, m ~ U{32..512}, n = m U{16..64},
                             l = 4m, k ~ U{1..64}, sigma 1 -> 1e-6; grouped
                             launches in a HIP graph against a loop of plans
  ipm_1024x131072            A (1024 x 131072, sigma 1 -> 1e-4) rescaled as
                             A D_t for 32 steps, l=4096, k=128 per step, all
                             steps batched against a step-by-step loop

value = projections per second = (right-hand sides) / (seconds per step),
inputs resident in HBM.  Prints one JSON line with the roofline of the
dominant stage (timed with HIP events on the plan's stream during the timed
steps), every form's errors against the CPU oracle on sampled right-hand
sides (refined and unrefined), and the oracle's own time on that sample as
the CPU baseline.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "projections/sec (Zb, k RHS) mixed vs FP64 at ≤1e-10 rel err; % HBM/MFMA peak"
TOL = 1e-10

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6          # matrix and vector (FMA = 2 flops)
PEAK_FP32_TFLOPS = 157.3         # MFMA binary32
PEAK_BF16_TFLOPS = 2500.0        # MFMA bfloat16, dense
PEAK_FP64_VALU_TOPS = 39.3       # FP64 VALU instructions/s: 256 CU x 64 lanes x 2.4 GHz
PEAK_INT8_TOPS = 5000.0          # MFMA int8, dense
# digit pairs the integer compensated products multiply: 11 signed base-128
# digits per operand (s, t = 0..10), pairs with s + t <= 11
OZ_PAIRS = sum(1 for s_ in range(11) for t_ in range(11) if s_ + t_ <= 11)
COMP_INT8 = 2

PRECISIONS = {"fp64": 0, "mixed_fp32": 1, "mixed_bf16": 2, "mixed_bf16x3": 3}


def log(msg):
    """Progress on stderr (the JSON result is the only stdout line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def stage_work(name, dims, prec="fp64", w_bits=64, inv=(2, 0), comp=1):
    """Algorithmic work per launch of a stage summed over the problems in
    `dims` (a list of (m, n, l, k)): (bound, amount, kind, peak).  `inv` is
    (method, iterations) of the Gram's inverse: 1 Newton-Schulz, 2 Cholesky;
    `comp` the form of the compensated products: 1 Dot2, 2 int8 digits."""
    tot = 0.0
    ns = inv[0] == 1
    int8 = comp == COMP_INT8 and name in ("refine_atx", "refine_ab")
    # plain products take the MFMA form for every problem once the largest
    # k reaches 32 (a batch decides for all its members at once)
    mfma_k = max(d[3] for d in dims) >= 32
    for (m, n, l, k) in dims:
        if name == "sketch":
            tot += 8.0 * m * n + 8.0 * m * l                               # read A, write S
        elif name == "qrcp":
            tot += 2.0 * l * m * m - 2.0 * m ** 3 / 3
        elif name == "qr_r0":
            # shifted Cholesky QR and one more pass: two Grams m(m+1)l, one
            # solve m^2 l, two Cholesky m^3/3, one triangular inverse m^3/3
            # and one triangular product m^3/3
            tot += 2.0 * m * (m + 1) * l + 1.0 * m * m * l + 4.0 * m ** 3 / 3
        elif name == "rinv_trsm":
            tot += m ** 3 / 3.0
        elif name == "gram_inv":
            tot += 4.0 * m ** 3 * inv[1] if ns else m ** 3 / 3.0        # two m^3 products per step
        elif name == "minv_form":
            tot += 24.0 * m * m if ns else m ** 3 / 3.0                  # R^{-T} Pi and its transpose
        elif name == "w_gemm":
            tot += 1.0 * m * m * n                                          # triangular: m^2 n
        elif name == "gram_syrk":
            tot += 1.0 * m * (m + 1) * n
        elif name in ("ab", "refine_atx_plain", "refine_ab_plain", "final_atx_plain"):
            if mfma_k:
                tot += 2.0 * m * n * k                                      # MFMA GEMM flops
            else:
                tot += 8.0 * m * n + 8.0 * n * k                            # read A and B (or x and r)
        elif int8:
            tot += OZ_PAIRS * 2.0 * m * n * k                               # int8 products of digit pairs
        elif name in ("refine_atx", "refine_ab", "final_atx"):
            tot += 10.0 * m * n * k                                         # Dot2: 10 FP64 ops per term
        else:
            return None, 0.0, None, None
    plain_pass = name in ("refine_atx_plain", "refine_ab_plain", "final_atx_plain")
    if name == "sketch" or (name == "minv_form" and ns) or ((plain_pass or name == "ab") and not mfma_k):
        return "hbm", tot, "bytes", PEAK_HBM_GBS
    if name == "qrcp":
        return "alu", tot, "flops", PEAK_FP64_TFLOPS
    if int8:
        return "mfma", tot, "ops", PEAK_INT8_TOPS
    if name in ("refine_atx", "refine_ab", "final_atx"):
        return "alu", tot, "ops", PEAK_FP64_VALU_TOPS
    if name == "gram_syrk" and prec == "mixed_bf16":
        return "mfma", tot, "flops", PEAK_BF16_TFLOPS
    if name == "gram_syrk" and prec == "mixed_fp32":
        return "mfma", tot, "flops", PEAK_FP32_TFLOPS
    if name == "gram_syrk" and prec == "mixed_bf16x3":
        return "mfma", 3.0 * tot, "flops", PEAK_BF16_TFLOPS                # three bfloat16 products
    if name == "w_gemm" and w_bits == 32:
        return "mfma", tot, "flops", PEAK_FP32_TFLOPS
    return "mfma", tot, "flops", PEAK_FP64_TFLOPS


# stage -> (kernel name in the profiler's trace, source file of that kernel)
STAGE_KERNELS = {
    "qrcp": ("qrcp_reg_kernel", "paper_0912_1135_amd/csrc/rt_qrcp.hip"),
    "sketch": ("sketch_pass", "paper_0912_1135_amd/csrc/rt_sketch.hip"),
    "gram_syrk": ("gemm_f64_kernel", "paper_0912_1135_amd/csrc/rt_gemm.hip"),
    "w_gemm": ("gemm_f64_kernel", "paper_0912_1135_amd/csrc/rt_gemm.hip"),
    "gram_inv": ("gemm_f64_kernel", "paper_0912_1135_amd/csrc/rt_gemm.hip"),
    "refine_atx": ("atx_kernel", "paper_0912_1135_amd/csrc/rt_apply.hip"),
    "final_atx": ("atx_kernel", "paper_0912_1135_amd/csrc/rt_apply.hip"),
    "refine_ab": ("ab_partial_kernel", "paper_0912_1135_amd/csrc/rt_apply.hip"),
}


def measured_traffic(stage, workload):
    """HBM bytes per launch of `stage`'s kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when there is
    none for this workload or the kernel's source changed since it was taken."""
    if stage not in STAGE_KERNELS:
        return None
    kernel, src = STAGE_KERNELS[stage]
    path = os.path.join(ROOT, "profiles", "traffic.md")
    try:
        text = open(path).read()
        digest = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()
    except OSError:
        return None
    for line in text.splitlines():
        if not line.startswith("traffic:"):
            continue
        kv = dict(re.findall(r"(\w+)=(\S+)", line))
        if kv.get("stage") == stage and kv.get("workload") == workload and kv.get("sha256") == digest:
            return float(kv["bytes_per_launch"])
    return None


def copy_calibration(mib):
    """One plain streaming kernel of known size (reads and writes `mib` MiB),
    the scale for the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    x = torch.ones(mib << 17, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    torch.neg(x, out=y)
    torch.cuda.synchronize()
    del x, y


def stage_table(info, steps, dims, prec, w_bits):
    stages = {}
    for name, tot in info["stage_ms"].items():
        calls = info["stage_calls"][name]
        if not calls:
            continue
        d = {"ms_per_step": tot / steps, "ms_per_launch": tot / calls, "launches_per_step": calls / steps}
        # the split-bfloat16 precision takes the binary32 Gram when n % 4 != 0
        gp = "mixed_fp32" if prec == "mixed_bf16x3" and info.get("gram_bits") == 32 else prec
        bound, amt, kind, peak = stage_work(name, dims, gp, w_bits,
                                            (info.get("inverse", 2), info.get("inverse_iters", 0)),
                                            info.get("comp_method", 1))
        if bound is not None:
            sec = d["ms_per_launch"] / 1e3
            if bound == "hbm":
                d["achieved"], d["unit"] = amt / sec / 1e9, "GB/s"
            else:
                d["achieved"], d["unit"] = amt / sec / 1e12, ("TOP/s" if kind == "ops" else "TFLOP/s")
            d["bound"], d["peak"], d["frac"] = bound, peak, d["achieved"] / peak
        stages[name] = d
    return stages


def roofline(stages, workload):
    dom = max(stages, key=lambda s: stages[s]["ms_per_step"])
    d = stages[dom]
    if "bound" not in d:
        return {"bound": None, "achieved": None, "peak": None, "unit": None, "frac": None, "traffic": None,
                "kernel": dom}
    return {"bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"], "unit": d["unit"],
            "frac": d["frac"], "traffic": measured_traffic(dom, workload), "kernel": dom}


def rel_errors(B, Z, Y, X, Zr, Yr, Xr):
    """max over right-hand sides (rows) of |z - z*|/|b|, |p - p*|/|b|, |x - x*|/|x*|."""
    import numpy as np
    nb = np.linalg.norm(B, axis=1)
    return (float(np.max(np.linalg.norm(Z - Zr, axis=1) / nb)),
            float(np.max(np.linalg.norm(Y - Yr, axis=1) / nb)),
            float(np.max(np.linalg.norm(X - Xr, axis=1) / np.linalg.norm(Xr, axis=1))))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def time_plan(plan, At, Bt, Z, Y, X, steps, warmup):
    import torch
    for _ in range(warmup):
        plan.precondition(At)
        plan.project_all(Bt, Z, Y, X)
    torch.cuda.synchronize()
    plan.set_timing(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        plan.precondition(At)
        plan.project_all(Bt, Z, Y, X)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    info = plan.info()
    plan.set_timing(False)
    return (t2 - t1) * 1e3 / steps, info


def run_single(args, rt, synth, np, torch):
    c = synth.CONFIGS[args.workload]
    m, n, l, k, kappa, seed = c["m"], c["n"], c["l"], c["k"], c["kappa"], c["seed"]
    t0 = time.time()
    log(f"generating {args.workload}: {m} x {n}")
    A = synth.make_problem(m, n, kappa, seed)
    B = synth.make_rhs(n, k, seed)
    gen_s = time.time() - t0
    log(f"inputs ready in {gen_s:.1f} s")
    dev = torch.device("cuda", 0)
    At = torch.from_numpy(A).to(dev)
    Bt = torch.from_numpy(B).to(dev)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
    mixed_wl = args.workload.startswith("mixed")
    main_prec = args.precision or ("mixed_bf16x3" if mixed_wl else "fp64")
    forms_to_run = [main_prec] + ([] if args.no_forms else [p for p in PRECISIONS if p != main_prec])
    dims = [(m, n, l, k)]
    forms, outputs, unrefined, main = {}, {}, {}, None
    # right-hand sides the oracle checks: all 16 of the 512 x 65536 workload
    # (one core each); one at larger sizes, where the oracle's factorization
    # of A^T alone takes about a minute
    big = m * n > 512 * 65536
    ks = min(k, 16) if not big else 1
    for prec in forms_to_run:
        plan = rt.Plan(m, n, l, seed)
        plan.set_precision(PRECISIONS[prec])
        plan.set_refinement(args.refine_steps, 0.0)
        plan.set_qr(args.qr)
        plan.set_inverse(args.inverse)
        plan.set_autotune(not args.no_autotune)  # new shapes are tuned in the warm-up steps
        Z, Y = torch.empty_like(Bt), torch.empty_like(Bt)
        X = torch.empty((k, m), dtype=torch.float64, device=dev)
        steps = args.steps if prec == main_prec else min(args.steps, args.form_steps)
        ms, info = time_plan(plan, At, Bt, Z, Y, X, steps, args.warmup)
        log(f"{prec}: {ms:.3f} ms per step")
        plan.status()  # raises if the refinement did not converge
        # the same preconditioner, unrefined, on the sampled right-hand sides
        plan.set_refinement(0, 0.0)
        unrefined[prec] = [t.cpu().numpy() for t in plan.project_all(Bt[:ks])]
        plan.close()
        stages = stage_table(info, steps, dims, prec, info["w_bits"])
        outputs[prec] = (Z.cpu().numpy(), Y.cpu().numpy(), X.cpu().numpy())
        forms[prec] = {"value": k / (ms / 1e3), "ms_per_step": ms, "steps": steps,
                       "refine_steps": info["refine_steps"], "refine_plain": info["refine_plain"],
                       "refine_comp": info["refine_comp"], "refine_err_est": info["refine_err_est"],
                       "sketch_bits": info["sketch_bits"],
                       "w_bits": info["w_bits"], "gram_bits": info["gram_bits"],
                       "sketch_escalated": info["sketch_escalated"], "kappa_est": info["kappa_est"],
                       "gram_cond_est": info["gram_cond_est"], "qr_mode": info["qr_mode"],
                       "inverse": info["inverse"], "inverse_iters": info["inverse_iters"],
                       "inverse_resid": info["inverse_resid"],
                       "stage_ms": {s: round(d["ms_per_step"], 4) for s, d in stages.items()}}
        if prec == main_prec:
            main = (ms, info, stages, steps)
        del Z, Y, X
    ms_per_step, info, stages, steps = main
    value = k / (ms_per_step / 1e3)
    paper = None if args.no_forms else paper_columns(rt, torch, np, At, Bt, m, n, l, k, seed, kappa, main_prec)
    bits = {"fp64": "f64", "mixed_fp32": "f64+f32", "mixed_bf16": "f64+bf16", "mixed_bf16x3": "f64+f32+bf16x3"}[main_prec]
    result = {
        "metric": METRIC, "value": value, "unit": "projections/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": bits, "data": "synthetic",
        "config": {"workload": f"{args.workload}: A = U diag(sigma) V^T (Haar U, V), m={m}, n={n}, "
                               f"sigma log-spaced 1..1/{kappa:g}, l={l}, k={k} Gaussian right-hand sides, "
                               f"{main_prec}", "m": m, "n": n, "l": l, "k": k, "kappa": kappa,
                   "precision": main_prec, "refine_steps": info["refine_steps"], "parallelism": "single GPU"},
        "roofline": roofline(stages, args.workload),
        "stages": stages,
        "forms": forms,
        "kappa_est": info["kappa_est"],
        "qrcp_blocks": info["qrcp_blocks"],
        "qr_mode": info["qr_mode"],
    }
    if main_prec != "fp64" and "fp64" in forms:
        result["mixed_vs_fp64"] = forms[main_prec]["value"] / forms["fp64"]["value"]
    if paper is not None:
        result["paper_columns"] = paper
    if not args.no_autotune:
        import tempfile
        with tempfile.TemporaryDirectory() as td:
            rt.autotune_save(os.path.join(td, "tune.txt"))
            result["autotune"] = [ln.split() for ln in open(os.path.join(td, "tune.txt")) if ln.strip()]
    # parity of every form against the oracle on the sampled right-hand sides
    # (refined and unrefined results); the oracle's time on that sample is the
    # CPU baseline.  Above 512 x 65536 the oracle takes R from LAPACK's
    # Householder QR of A^T (its unblocked factorization would take minutes).
    cpu_sample = None
    if not (args.no_parity and args.no_cpu_baseline):
        import oracle
        threads = oracle.num_threads()
        route = oracle.project_lapack if big else oracle.project
        log(f"oracle on {ks} right-hand side(s)")
        t3 = time.perf_counter()
        Zr, Yr, Xr, _ = route(A, B[:ks].T)
        t4 = time.perf_counter()
        log(f"oracle done in {t4 - t3:.1f} s")
        for prec, (Zg, Yg, Xg) in outputs.items():
            ez, ep, ex = rel_errors(B[:ks], Zg[:ks], Yg[:ks], Xg[:ks], Zr.T, Yr.T, Xr.T)
            u = rel_errors(B[:ks], *unrefined[prec], Zr.T, Yr.T, Xr.T)
            forms[prec].update({"e_z": ez, "e_p": ep, "e_x": ex, "parity": "oracle", "columns_checked": ks,
                                "unrefined_e_z": u[0], "unrefined_e_p": u[1], "unrefined_e_x": u[2],
                                "pass": max(ez, ep, ex) <= TOL})
        if not args.no_cpu_baseline:
            how = ("Householder QR of A^T (LAPACK, R only) plus binary128 refinement" if big else
                   "Householder QR of A^T plus binary128 refinement")
            cpu_sample = {"value": ks / (t4 - t3), "unit": "projections/s", "cores": threads, "kind": "oracle",
                          "cpu_model": cpu_model(),
                          "sample": f"{how} for {ks} of the {k} right-hand sides of the same {m} x {n} workload "
                                    f"({t4 - t3:.1f} s)"}
    if big and "fp64" in outputs:
        # every column: against the binary64 form
        Z64, Y64, X64 = outputs["fp64"]
        for prec, (Zg, Yg, Xg) in outputs.items():
            ez, ep, ex = rel_errors(B, Zg, Yg, Xg, Z64, Y64, X64)
            forms[prec].update({"e_z_vs_fp64": ez, "e_p_vs_fp64": ep, "e_x_vs_fp64": ex})
    result["cpu_baseline"] = cpu_sample
    result["parity"] = {p: {key: forms[p][key] for key in ("e_z", "e_p", "e_x", "unrefined_e_z", "unrefined_e_p",
                                                           "unrefined_e_x", "e_z_vs_fp64", "e_p_vs_fp64",
                                                           "e_x_vs_fp64", "pass") if key in forms[p]}
                        for p in forms}
    result["input_generation_s"] = gen_s
    return result


def paper_columns(rt, torch, np, At, Bt, m, n, l, k, seed, kappa, main_prec):
    """The columns of the paper's tables (Sec. 5) on this workload: s_pre and
    s_pro of the classical scheme (A A^T, its pivoted QR, then eq.
    basic_identity per right-hand side), t_pre and t_pro of the randomized
    method, and delta = max |A z|, epsilon = max |Z z - z| over 8 random unit
    vectors b, divided by cond(A) as the tables report them."""
    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps
    Bu = Bt[:8] / torch.linalg.vector_norm(Bt[:8], dim=1, keepdim=True)
    out = {}
    for name, method, prec, steps in [("classical", rt.METHOD_CLASSICAL, "fp64", -1),
                                      ("randomized_unrefined", rt.METHOD_RANDOMIZED, "fp64", 0),
                                      ("randomized", rt.METHOD_RANDOMIZED, main_prec, -1),
                                      ("randomized_krylov", rt.METHOD_KRYLOV, "fp64", -1)]:
        plan = rt.Plan(m, n, l, seed)
        plan.set_method(method)
        plan.set_precision(PRECISIONS[prec])
        plan.set_refinement(steps, 0.0)
        t_pre = timed(lambda: plan.precondition(At))
        Z = torch.empty_like(Bt)
        t_pro = timed(lambda: plan.project_null(Bt, out=Z)) / k
        Zu = plan.project_null(Bu)
        ZZ = plan.project_null(Zu)
        torch.cuda.synchronize()
        delta = torch.linalg.vector_norm(Zu @ At.T, dim=1).max().item()
        eps = torch.linalg.vector_norm(ZZ - Zu, dim=1).max().item()
        out[name] = {"pre_s": t_pre, "pro_s": t_pro, "delta_over_kappa": delta / kappa,
                     "epsilon_over_kappa": eps / kappa, "precision": prec}
        log(f"{name}: pre {t_pre * 1e3:.2f} ms, pro {t_pro * 1e6:.1f} us per rhs, "
            f"delta/kappa {delta / kappa:.2e}, epsilon/kappa {eps / kappa:.2e}")
        plan.close()
    return out


def run_paper(args, rt, synth, np, torch):
    """The paper's Table 1 / Table 2 workload (Sec. 5, eq. test_mat): A =
    U [B ... B] V with m = 400, n = 1e6, l = 404, cond(A) = 1e8, G drawn as
    lagged-Fibonacci uniform [-1, 1] (passed in), k = 8 random unit vectors.
    Both schemes' columns: s_pre, s_pro (classical), t_pre, t_pro
    (randomized), delta / kappa and epsilon / kappa; z and A^T x against the
    exact block-average projection for every right-hand side."""
    from oracle.paper_forms import block_average_projection
    c = synth.CONFIGS[args.workload]
    m, n, l, k, kappa, seed = c["m"], c["n"], c["l"], c["k"], c["kappa"], c["seed"]
    log(f"generating {args.workload}")
    t0 = time.time()
    A, rp, cp = synth.make_paper_matrix(m, n, kappa, seed)
    G = synth.make_lfg_sketch(n, l, seed)
    B = synth.make_rhs(n, k, seed)
    B /= np.linalg.norm(B, axis=1, keepdims=True)
    gen_s = time.time() - t0
    log(f"inputs ready in {gen_s:.1f} s")
    dev = torch.device("cuda", 0)
    At, Gt, Bt = (torch.from_numpy(x).to(dev) for x in (A, G, B))
    Zc, Pc = block_average_projection(m, cp, B.T)
    nb = np.linalg.norm(B, axis=1)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps
    rows = {}
    for name, method, sketch in [("classical", rt.METHOD_CLASSICAL, None), ("randomized_lfg", rt.METHOD_RANDOMIZED, Gt),
                                 ("randomized_srft", rt.METHOD_RANDOMIZED, None)]:
        plan = rt.Plan(m, n, l, seed)
        plan.set_method(method)
        if sketch is not None:
            plan.set_sketch_matrix(sketch)
        pre = timed(lambda: plan.precondition(At), args.steps)
        Z = torch.empty_like(Bt)
        pro = timed(lambda: plan.project_null(Bt, out=Z), args.steps) / k
        ZZ = plan.project_null(Z)
        torch.cuda.synchronize()
        delta = torch.linalg.vector_norm(Z @ At.T, dim=1).max().item()
        eps = torch.linalg.vector_norm(ZZ - Z, dim=1).max().item()
        ez = float(np.max(np.linalg.norm(Z.cpu().numpy() - Zc.T, axis=1) / nb))
        rows[name] = {"pre_s": pre, "pro_s": pro, "delta_over_kappa": delta / kappa, "epsilon_over_kappa": eps / kappa,
                      "e_z_vs_closed_form": ez, "kappa_est": plan.info()["kappa_est"]}
        log(f"{name}: pre {pre * 1e3:.2f} ms, pro {pro * 1e6:.1f} us per vector, delta/kappa {delta / kappa:.2e}, "
            f"epsilon/kappa {eps / kappa:.2e}, e_z {ez:.2e}")
        plan.close()
    r = rows["randomized_lfg"]
    ms = (r["pre_s"] + k * r["pro_s"]) * 1e3
    value = k / (ms / 1e3)
    return {
        "metric": METRIC, "value": value, "unit": "projections/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: A = U [B ... B] V (eq. test_mat), m={m}, n={n}, l={l}, "
                               f"cond {kappa:g}, lagged-Fibonacci G, {k} random unit vectors",
                   "m": m, "n": n, "l": l, "k": k, "kappa": kappa, "parallelism": "single GPU"},
        "paper_columns": rows,
        "parity": {"e_z_vs_closed_form": r["e_z_vs_closed_form"], "pass": r["e_z_vs_closed_form"] <= TOL},
        "cpu_baseline": None,
        "input_generation_s": gen_s,
    }


def run_complex(args, rt, synth, np, torch):
    """Complex A (the paper's extension to complex entries, Sec. 1): a
    complex m x n A = U diag(sigma) V^* projected through the real embedding
    (rtproj_cplan_*), against the complex oracle on two right-hand sides."""
    from oracle import complex_oracle
    c = synth.CONFIGS[args.workload]
    m, n, l, k, kappa, seed = c["m"], c["n"], c["l"], c["k"], c["kappa"], c["seed"]
    log(f"generating {args.workload}")
    A = synth.make_complex_problem(m, n, kappa, seed)
    B = synth.make_complex_rhs(n, k, seed)
    dev = torch.device("cuda", 0)
    At, Bt = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
    plan = rt.CPlan(m, n, l, seed)
    Z, Y, X = torch.empty_like(Bt), torch.empty_like(Bt), torch.empty((k, m), dtype=Bt.dtype, device=dev)
    for _ in range(args.warmup):
        plan.precondition(At)
        plan.project_all(Bt, Z, Y, X)
    torch.cuda.synchronize()
    plan.real.set_timing(True)
    t1 = time.perf_counter()
    for _ in range(args.steps):
        plan.precondition(At)
        plan.project_all(Bt, Z, Y, X)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t1) * 1e3 / args.steps
    info = plan.real.info()
    plan.real.status()
    stages = stage_table(info, args.steps, [(2 * m, 2 * n, 2 * l, k)], "fp64", 64)
    t3 = time.perf_counter()
    Zr, Yr, Xr, _ = complex_oracle.project_complex(A, B[:2].T)
    t4 = time.perf_counter()
    ez, ep, ex = rel_errors(B[:2], Z[:2].cpu().numpy(), Y[:2].cpu().numpy(), X[:2].cpu().numpy(), Zr.T, Yr.T, Xr.T)
    plan.close()
    return {
        "metric": METRIC, "value": k / (ms / 1e3), "unit": "projections/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c128 (as f64 real embedding)", "data": "synthetic",
        "config": {"workload": f"{args.workload}: complex A = U diag(sigma) V^*, m={m}, n={n}, l={l}, "
                               f"sigma 1..1/{kappa:g}, k={k}; real 2m x 2n embedding", "m": m, "n": n, "l": l,
                   "k": k, "kappa": kappa, "parallelism": "single GPU"},
        "roofline": roofline(stages, args.workload), "stages": stages,
        "parity": {"e_z": ez, "e_p": ep, "e_x": ex, "columns_checked": 2, "pass": max(ez, ep, ex) <= TOL},
        "cpu_baseline": {"value": 2 / (t4 - t3), "unit": "projections/s", "cores": len(os.sched_getaffinity(0)),
                         "kind": "oracle", "cpu_model": cpu_model(),
                         "sample": f"complex oracle on 2 of the {k} right-hand sides ({t4 - t3:.1f} s)"},
    }


def run_batch(args, rt, synth, np, torch):
    c = synth.CONFIGS[args.workload]
    count, kappa, seed = c["count"], c["kappa"], c["seed"]
    shp = synth.make_batch_shapes(count, seed)
    t0 = time.time()
    log(f"generating {count} members")
    As = []
    for i, (m, n) in enumerate(zip(shp.m, shp.n)):
        As.append(synth.make_problem(m, n, kappa, seed + 1000 + i))
        if i % 64 == 63:
            log(f"  {i + 1} members")
    Bs = [synth.make_rhs(n, k, seed + 5000 + i) for i, (n, k) in enumerate(zip(shp.n, shp.k))]
    gen_s = time.time() - t0
    log(f"inputs ready in {gen_s:.1f} s")
    dev = torch.device("cuda", 0)
    At = [torch.from_numpy(A).to(dev) for A in As]
    Bt = [torch.from_numpy(B).to(dev) for B in Bs]
    Z = [torch.empty_like(b) for b in Bt]
    Y = [torch.empty_like(b) for b in Bt]
    X = [torch.empty((k, m), dtype=torch.float64, device=dev) for m, k in zip(shp.m, shp.k)]
    ksum = int(sum(shp.k))
    dims = list(zip(shp.m, shp.n, shp.l, shp.k))
    bt = rt.Batch(shp.m, shp.n, shp.l, seed)
    # per-stage times from eager (ungraphed) steps
    bt.set_graph(False)
    bt.precondition(At)
    bt.project_all(Bt, Z, Y, X)
    torch.cuda.synchronize()
    bt.set_timing(True)
    tsteps = 2
    for _ in range(tsteps):
        bt.precondition(At)
        bt.project_all(Bt, Z, Y, X)
    torch.cuda.synchronize()
    binfo = bt.info()
    bt.set_timing(False)
    stages = stage_table(binfo, tsteps, dims, "fp64", 64)
    # the timed steps replay the captured graphs
    bt.set_graph(True)
    for _ in range(args.warmup):
        bt.precondition(At)
        bt.project_all(Bt, Z, Y, X)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        bt.precondition(At)
        bt.project_all(Bt, Z, Y, X)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    status = bt.status()
    ms_per_step = (t2 - t1) * 1e3 / args.steps
    log(f"batch (graph): {ms_per_step:.3f} ms per step")
    # the same batch with the binary32 grouped Gram
    bt.set_precision(1)
    for _ in range(args.warmup):
        bt.precondition(At)
        bt.project_all(Bt, Z, Y, X)
    torch.cuda.synchronize()
    t1b = time.perf_counter()
    for _ in range(args.steps):
        bt.precondition(At)
        bt.project_all(Bt, Z, Y, X)
    torch.cuda.synchronize()
    ms32 = (time.perf_counter() - t1b) * 1e3 / args.steps
    status32 = bt.status()
    log(f"batch (graph, binary32 Gram): {ms32:.3f} ms per step")
    # and with the split-bfloat16 grouped Gram (its outputs are the ones
    # checked against the oracle below)
    bt.set_precision(3)
    for _ in range(args.warmup):
        bt.precondition(At)
        bt.project_all(Bt, Z, Y, X)
    torch.cuda.synchronize()
    t1c = time.perf_counter()
    for _ in range(args.steps):
        bt.precondition(At)
        bt.project_all(Bt, Z, Y, X)
    torch.cuda.synchronize()
    msx3 = (time.perf_counter() - t1c) * 1e3 / args.steps
    statusx3 = bt.status()
    log(f"batch (graph, split-bfloat16 Gram): {msx3:.3f} ms per step")
    value = ksum / (ms_per_step / 1e3)
    # baseline on the same GPU: one binary64 plan per member, one after another
    plans = [rt.Plan(m, n, l, 0) for m, n, l in zip(shp.m, shp.n, shp.l)]
    Zl = [torch.empty_like(b) for b in Bt]
    for p, a, b, z in zip(plans, At, Bt, Zl):  # warm-up
        p.precondition(a)
        p.project_all(b, z, None, None, want=(True, False, False))
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for p, a, b, z in zip(plans, At, Bt, Zl):
        p.precondition(a)
        p.project_all(b, z, None, None, want=(True, False, False))
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    for p in plans:
        p.close()
    loop_value = ksum / (t4 - t3)
    log(f"loop of plans: {(t4 - t3) * 1e3:.3f} ms per step")
    result = {
        "metric": METRIC, "value": value, "unit": "projections/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {count} members, m ~ U{{32..512}}, n = m U{{16..64}}, l = 4m, "
                               f"k ~ U{{1..64}}, sigma log-spaced 1..1/{kappa:g}; grouped launches replayed from "
                               "a HIP graph", "members": count, "sum_k": ksum,
                   "sum_mn": int(sum(m * n for m, n in zip(shp.m, shp.n))), "precision": "fp64",
                   "refine_steps": binfo["refine_steps"], "parallelism": "single GPU"},
        "roofline": roofline(stages, args.workload),
        "stages": stages,
        "forms": {"batch_graph": {"value": value, "ms_per_step": ms_per_step},
                  "batch_graph_fp32_gram": {"value": ksum / (ms32 / 1e3), "ms_per_step": ms32,
                                            "member_status_nonzero": [i for i, s in enumerate(status32) if s != 0]},
                  "batch_graph_bf16x3_gram": {"value": ksum / (msx3 / 1e3), "ms_per_step": msx3,
                                              "member_status_nonzero": [i for i, s in enumerate(statusx3)
                                                                        if s != 0]},
                  "loop_of_plans": {"value": loop_value, "ms_per_step": (t4 - t3) * 1e3}},
        "member_status_nonzero": [i for i, s in enumerate(status) if s != 0],
    }
    cpu_sample = None
    if not (args.no_parity and args.no_cpu_baseline):
        import oracle
        threads = oracle.num_threads()
        order = np.argsort(np.array(shp.m) * np.array(shp.n))
        pick = sorted(set([int(order[0]), int(order[len(order) // 2]), int(order[-1])] +
                          [int(i) for i in np.linspace(0, count - 1, 5).astype(int)]))
        worst = [0.0, 0.0, 0.0]
        t5 = time.perf_counter()
        kdone = 0
        log(f"oracle on members {pick}")
        for i in pick:
            Zr, Yr, Xr, _ = oracle.project(As[i], Bs[i].T)
            kdone += Bs[i].shape[0]
            e = rel_errors(Bs[i], Z[i].cpu().numpy(), Y[i].cpu().numpy(), X[i].cpu().numpy(), Zr.T, Yr.T, Xr.T)
            worst = [max(a, b) for a, b in zip(worst, e)]
        t6 = time.perf_counter()
        result["parity"] = {"members_checked": pick, "e_z": worst[0], "e_p": worst[1], "e_x": worst[2],
                            "tol": TOL, "pass": max(worst) <= TOL, "form": "batch_graph_bf16x3_gram (last run)"}
        if not args.no_cpu_baseline:
            cpu_sample = {"value": kdone / (t6 - t5), "unit": "projections/s", "cores": threads, "kind": "oracle",
                          "sample": f"members {pick} of the same batch (all their right-hand sides, "
                                    f"{kdone} projections, {t6 - t5:.1f} s)"}
    result["cpu_baseline"] = cpu_sample
    result["input_generation_s"] = gen_s
    bt.close()
    return result


def run_ipm(args, rt, synth, np, torch):
    """Interior-point-shaped sequence: a fixed A rescaled as A D_t for every
    step t, preconditioner rebuilt and k right-hand sides projected per step,
    all steps in one batch (grouped launches, HIP graph) against a loop over
    the steps with one binary64 plan."""
    c = synth.CONFIGS[args.workload]
    m, n, l, k, steps, kappa, seed = c["m"], c["n"], c["l"], c["k"], c["steps"], c["kappa"], c["seed"]
    log(f"generating {args.workload}: base {m} x {n}, {steps} scalings, {k} right-hand sides per step")
    t0 = time.time()
    A = synth.make_problem(m, n, kappa, seed)
    D = synth.make_scalings(n, steps, seed)
    dev = torch.device("cuda", 0)
    At = torch.from_numpy(A).to(dev)
    Dt = [torch.from_numpy(np.ascontiguousarray(D[t])).to(dev) for t in range(steps)]
    Bt = [torch.from_numpy(synth.make_rhs(n, k, seed + 100 + t)).to(dev) for t in range(steps)]
    gen_s = time.time() - t0
    log(f"inputs ready in {gen_s:.1f} s")
    Z = [torch.empty_like(b) for b in Bt]
    Y = [torch.empty_like(b) for b in Bt]
    X = [torch.empty((k, m), dtype=torch.float64, device=dev) for _ in range(steps)]
    dims = [(m, n, l, k)] * steps
    bt = rt.Batch([m] * steps, [n] * steps, [l] * steps, seed)
    bt.set_graph(False)
    bt.precondition([At] * steps, Dt)
    bt.project_all(Bt, Z, Y, X)
    torch.cuda.synchronize()
    bt.set_timing(True)
    bt.precondition([At] * steps, Dt)
    bt.project_all(Bt, Z, Y, X)
    torch.cuda.synchronize()
    binfo = bt.info()
    stages = stage_table(binfo, 1, dims, "fp64", 64)
    bt.set_timing(False)
    bt.set_graph(True)
    for _ in range(args.warmup):
        bt.precondition([At] * steps, Dt)
        bt.project_all(Bt, Z, Y, X)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        bt.precondition([At] * steps, Dt)
        bt.project_all(Bt, Z, Y, X)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    status = bt.status()
    ms_per_step = (t2 - t1) * 1e3 / args.steps
    value = steps * k / (ms_per_step / 1e3)
    log(f"batch of {steps} steps (graph): {ms_per_step:.1f} ms")
    # the same sequence with the binary32 grouped Gram
    bt.set_precision(1)
    for _ in range(args.warmup):
        bt.precondition([At] * steps, Dt)
        bt.project_all(Bt, Z, Y, X)
    torch.cuda.synchronize()
    t1b = time.perf_counter()
    for _ in range(args.steps):
        bt.precondition([At] * steps, Dt)
        bt.project_all(Bt, Z, Y, X)
    torch.cuda.synchronize()
    ms32 = (time.perf_counter() - t1b) * 1e3 / args.steps
    status32 = bt.status()
    refine32 = bt.info()["refine_steps"]
    log(f"batch of {steps} steps (graph, binary32 Gram): {ms32:.1f} ms, {refine32} refinement steps")
    # and with the split-bfloat16 grouped Gram (binary32 P^{-1}A); its
    # outputs are the ones checked against the oracle below
    bt.set_precision(3)
    for _ in range(args.warmup):
        bt.precondition([At] * steps, Dt)
        bt.project_all(Bt, Z, Y, X)
    torch.cuda.synchronize()
    t1c = time.perf_counter()
    for _ in range(args.steps):
        bt.precondition([At] * steps, Dt)
        bt.project_all(Bt, Z, Y, X)
    torch.cuda.synchronize()
    msx3 = (time.perf_counter() - t1c) * 1e3 / args.steps
    statusx3 = bt.status()
    refinex3 = bt.info()["refine_steps"]
    log(f"batch of {steps} steps (graph, split-bfloat16 Gram): {msx3:.1f} ms, {refinex3} refinement steps")
    # the sequential loop: one plan, A D_t formed on the device, step by step
    plan = rt.Plan(m, n, l, seed)
    Ad = torch.empty_like(At)
    Zl = torch.empty_like(Bt[0])
    torch.mul(At, Dt[0][None, :], out=Ad)
    plan.precondition(Ad)
    plan.project_all(Bt[0], Zl, None, None, want=(True, False, False))
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for t in range(steps):
        torch.mul(At, Dt[t][None, :], out=Ad)
        plan.precondition(Ad)
        plan.project_all(Bt[t], Zl, None, None, want=(True, False, False))
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    plan.close()
    loop_value = steps * k / (t4 - t3)
    log(f"loop of steps: {(t4 - t3) * 1e3:.1f} ms")
    result = {
        "metric": METRIC, "value": value, "unit": "projections/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: base A = U diag(sigma) V^T, m={m}, n={n}, sigma log-spaced "
                               f"1..1/{kappa:g}, rescaled A D_t for {steps} steps with D_t = diag(10^U(-6,6)); "
                               f"l={l}, k={k} right-hand sides per step; all steps batched, HIP graph",
                   "m": m, "n": n, "l": l, "k": k, "ipm_steps": steps, "precision": "fp64",
                   "refine_steps": binfo["refine_steps"],
                   "parallelism": "single GPU"},
        "roofline": roofline(stages, args.workload),
        "stages": stages,
        "forms": {"batch_graph": {"value": value, "ms_per_step": ms_per_step},
                  "batch_graph_fp32_gram": {"value": steps * k / (ms32 / 1e3), "ms_per_step": ms32,
                                            "refine_steps": refine32,
                                            "member_status_nonzero": [i for i, s_ in enumerate(status32) if s_ != 0]},
                  "batch_graph_bf16x3_gram": {"value": steps * k / (msx3 / 1e3), "ms_per_step": msx3,
                                              "refine_steps": refinex3,
                                              "member_status_nonzero": [i for i, s_ in enumerate(statusx3)
                                                                        if s_ != 0]},
                  "loop_of_steps": {"value": loop_value, "ms_per_step": (t4 - t3) * 1e3}},
        "member_status_nonzero": [i for i, s_ in enumerate(status) if s_ != 0],
    }
    cpu_sample = None
    if not (args.no_parity and args.no_cpu_baseline):
        import oracle
        threads = oracle.num_threads()
        worst = [0.0, 0.0, 0.0]
        t5 = time.perf_counter()
        pick = [0, steps - 1]
        for t in pick:
            log(f"oracle on step {t}")
            As = A * D[t][None, :]
            Bs = Bt[t][:2].cpu().numpy()
            Zr, Yr, Xr, _ = oracle.project(As, Bs.T)
            e = rel_errors(Bs, Z[t][:2].cpu().numpy(), Y[t][:2].cpu().numpy(), X[t][:2].cpu().numpy(),
                           Zr.T, Yr.T, Xr.T)
            worst = [max(a, b) for a, b in zip(worst, e)]
        t6 = time.perf_counter()
        result["parity"] = {"steps_checked": pick, "columns_per_step": 2, "e_z": worst[0], "e_p": worst[1],
                            "e_x": worst[2], "tol": TOL, "pass": max(worst) <= TOL,
                            "form": "batch_graph_bf16x3_gram (last run)"}
        if not args.no_cpu_baseline:
            cpu_sample = {"value": 2 * len(pick) / (t6 - t5), "unit": "projections/s", "cores": threads,
                          "kind": "oracle", "sample": f"2 right-hand sides of steps {pick} ({t6 - t5:.1f} s)"}
    result["cpu_baseline"] = cpu_sample
    result["input_generation_s"] = gen_s
    bt.close()
    return result


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mixed_2048x262144",
                    choices=["plain_512x65536", "plain_64x4096", "mixed_2048x262144", "batch_256",
                             "ipm_1024x131072", "paper_400x1000000", "complex_512x32768"])
    ap.add_argument("--precision", default=None, choices=list(PRECISIONS),
                    help="form of the main line (default: fp64, or mixed_bf16x3 for the mixed workload)")
    ap.add_argument("--no-forms", action="store_true", help="time only the main precision")
    ap.add_argument("--form-steps", type=int, default=10, help="timed steps of the other precision forms")
    ap.add_argument("--refine-steps", type=int, default=-1, help="-1: chosen from the pivoted-QR rank estimate")
    ap.add_argument("--qr", type=int, default=0, help="pivoted-QR method: 0 auto, 1 direct, 2 two-stage, "
                                                      "3 two-stage with a single-workgroup second stage")
    ap.add_argument("--inverse", type=int, default=0, help="Gram inverse: 0 auto, 1 Newton-Schulz, 2 Cholesky")
    ap.add_argument("--no-autotune", action="store_true", help="built-in GEMM configurations only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run one plain copy kernel over MIB MiB (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path; use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_0912_1135_amd as rt
    from paper_0912_1135_amd import synth

    if args.workload == "batch_256":
        result = run_batch(args, rt, synth, np, torch)
    elif args.workload.startswith("paper_"):
        result = run_paper(args, rt, synth, np, torch)
    elif args.workload.startswith("complex_"):
        result = run_complex(args, rt, synth, np, torch)
    elif args.workload == "ipm_1024x131072":
        result = run_ipm(args, rt, synth, np, torch)
    else:
        result = run_single(args, rt, synth, np, torch)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
