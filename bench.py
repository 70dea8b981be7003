#!/usr/bin/env python3
"""Throughput of the randomized orthogonal projection on one MI355X.

One step = the whole path on one batch: precondition A (sketch, pivoted QR,
R^{-T}, P^{-1}A, Gram, Cholesky) and project k right-hand sides (least squares
x, row projection A^T x, null projection b - A^T x, with the double-binary64
refinement), all through the C ABI.  The default workload is the binary64
one: m = 512, n = 65536, singular values log-spaced 1 -> 1e-10, l = 2048,
k = 16 Gaussian right-hand sides.

value = projections per second = k / (seconds per step), inputs resident in
HBM.  Prints one JSON line with the roofline of the dominant kernel (timed
with HIP events on the plan's stream during the timed steps) and the CPU
oracle timed on a bounded sample of the same workload.
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

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6          # matrix and vector (FMA = 2 flops)
PEAK_FP64_VALU_TOPS = 39.3       # FP64 VALU instructions/s: 256 CU x 64 lanes x 2.4 GHz


def stage_work(name, m, n, l, k, refine_steps):
    """Algorithmic work per launch of a stage: (bound, amount, unit-kind)."""
    if name == "sketch":
        return "hbm", 8.0 * m * n + 8.0 * m * l, "bytes"          # read A, write S
    if name == "qrcp":
        return "alu", 2.0 * l * m * m - 2.0 * m ** 3 / 3, "flops"
    if name == "qr_r0":
        # shifted Cholesky QR: three Grams (m(m+1) l), two solves (m^2 l),
        # three Cholesky (m^3/3) and two triangular products (m^3/3)
        return "mfma", 3.0 * m * (m + 1) * l + 2.0 * m * m * l + 5.0 * m ** 3 / 3, "flops"
    if name == "rinv_trsm":
        return "mfma", m ** 3 / 3.0, "flops"
    if name == "w_gemm":
        return "mfma", 1.0 * m * m * n, "flops"                    # triangular: m^2 n
    if name == "gram_syrk":
        return "mfma", 1.0 * m * (m + 1) * n, "flops"
    if name == "cholesky":
        return "mfma", m ** 3 / 3.0, "flops"
    if name == "t_trsm":
        return "mfma", m ** 3 / 3.0, "flops"
    if name == "ab":
        return "hbm", 8.0 * m * n + 8.0 * n * k, "bytes"           # read A and B
    if name in ("refine_atx", "refine_ab", "final_atx"):
        return "alu", 10.0 * m * n * k, "ops"                      # Dot2: 10 FP64 ops per term
    return None, 0.0, None


# stage -> (kernel name in the profiler's trace, source file of that kernel)
STAGE_KERNELS = {
    "qrcp": ("qrcp_kernel", "paper_0912_1135_amd/csrc/rt_qrcp.hip"),
    "sketch": ("sketch_pass", "paper_0912_1135_amd/csrc/rt_sketch.hip"),
    "gram_syrk": ("gemm_f64_kernel", "paper_0912_1135_amd/csrc/rt_gemm.hip"),
    "w_gemm": ("gemm_f64_kernel", "paper_0912_1135_amd/csrc/rt_gemm.hip"),
    "cholesky": ("chol_diag_kernel", "paper_0912_1135_amd/csrc/rt_factor.hip"),
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plain_512x65536",
                    help="plain_512x65536 or plain_64x4096 (single-instance binary64 workloads)")
    ap.add_argument("--refine-steps", type=int, default=-1, help="-1: chosen from the pivoted-QR rank estimate")
    ap.add_argument("--qr", type=int, default=0, help="pivoted-QR method: 0 auto, 1 direct, 2 two-stage, "
                                                      "3 two-stage with a single-workgroup second stage")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run one plain copy kernel over MIB MiB (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md); use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_0912_1135_amd as rt
    from paper_0912_1135_amd import synth

    c = synth.CONFIGS[args.workload]
    m, n, l, k, kappa, seed = c["m"], c["n"], c["l"], c["k"], c["kappa"], c["seed"]
    t0 = time.time()
    A = synth.make_problem(m, n, kappa, seed)
    B = synth.make_rhs(n, k, seed)
    gen_s = time.time() - t0
    dev = torch.device("cuda", 0)
    At = torch.from_numpy(A).to(dev)
    Bt = torch.from_numpy(B).to(dev)
    Z = torch.empty_like(Bt)
    Y = torch.empty_like(Bt)
    X = torch.empty((k, m), dtype=torch.float64, device=dev)

    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
    plan = rt.Plan(m, n, l, seed)
    plan.set_refinement(args.refine_steps, 0.0)
    plan.set_qr(args.qr)

    def step():
        plan.precondition(At)
        plan.project_all(Bt, Z, Y, X)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.set_timing(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    info = plan.info()
    plan.set_timing(False)
    ms_per_step = (t2 - t1) * 1e3 / args.steps
    value = k / (ms_per_step / 1e3)

    # per-stage device time per step and the dominant stage's roofline
    stages = {}
    for name, tot in info["stage_ms"].items():
        calls = info["stage_calls"][name]
        if calls:
            stages[name] = {"ms_per_step": tot / args.steps, "ms_per_launch": tot / calls,
                            "launches_per_step": calls / args.steps}
    dom = max(stages, key=lambda s: stages[s]["ms_per_step"])
    bound, amount, kind = stage_work(dom, m, n, l, k, args.refine_steps)
    sec = stages[dom]["ms_per_launch"] / 1e3
    if bound == "hbm":
        roof = {"bound": "hbm", "achieved": amount / sec / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    elif bound == "mfma":
        roof = {"bound": "mfma", "achieved": amount / sec / 1e12, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s"}
    elif kind == "ops":
        roof = {"bound": "alu", "achieved": amount / sec / 1e12, "peak": PEAK_FP64_VALU_TOPS, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "alu", "achieved": amount / sec / 1e12, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(dom, args.workload)
    roof["kernel"] = dom
    for name, d in stages.items():
        b, amt, kd = stage_work(name, m, n, l, k, args.refine_steps)
        if b is None:
            continue
        s = d["ms_per_launch"] / 1e3
        if b == "hbm":
            d["achieved"], d["unit"], d["frac"] = amt / s / 1e9, "GB/s", amt / s / 1e9 / PEAK_HBM_GBS
        elif kd == "ops":
            d["achieved"], d["unit"], d["frac"] = amt / s / 1e12, "TOP/s", amt / s / 1e12 / PEAK_FP64_VALU_TOPS
        else:
            d["achieved"], d["unit"], d["frac"] = amt / s / 1e12, "TFLOP/s", amt / s / 1e12 / PEAK_FP64_TFLOPS

    result = {
        "metric": METRIC, "value": value, "unit": "projections/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"fp64 plain: A = U diag(sigma) V^T, m={m}, n={n}, sigma log-spaced 1..1/{kappa:g}, "
                               f"l={l}, k={k} Gaussian RHS", "m": m, "n": n, "l": l, "k": k, "kappa": kappa,
                   "precision": "fp64", "refine_steps": info["refine_steps"], "parallelism": "single GPU"},
        "roofline": roof,
        "stages": stages,
        "kappa_est": info["kappa_est"],
        "qrcp_blocks": info["qrcp_blocks"],
        "qr_mode": info["qr_mode"],
    }

    cpu_sample = None
    if not args.no_parity or not args.no_cpu_baseline:
        import oracle
        threads = oracle.num_threads()
        ks = min(k, threads)
        Zg, Yg, Xg = Z[:ks].cpu().numpy(), Y[:ks].cpu().numpy(), X[:ks].cpu().numpy()
        t3 = time.perf_counter()
        Zr, Yr, Xr, oinfo = oracle.project(A, B[:ks].T)
        t4 = time.perf_counter()
        nb = np.linalg.norm(B[:ks], axis=1)
        result["parity"] = {
            "columns_checked": ks,
            "e_z": float(np.max(np.linalg.norm(Zg - Zr.T, axis=1) / nb)),
            "e_p": float(np.max(np.linalg.norm(Yg - Yr.T, axis=1) / nb)),
            "e_x": float(np.max(np.linalg.norm(Xg - Xr.T, axis=1) / np.linalg.norm(Xr.T, axis=1))),
            "tol": 1e-10,
        }
        if not args.no_cpu_baseline:
            cpu_sample = {"value": ks / (t4 - t3), "unit": "projections/s", "cores": threads, "kind": "oracle",
                          "sample": f"Householder QR of A^T plus binary128 refinement for {ks} of the {k} "
                                    f"right-hand sides of the same {m} x {n} workload ({t4 - t3:.1f} s)"}
    result["cpu_baseline"] = cpu_sample
    result["input_generation_s"] = gen_s
    plan.close()
    print(json.dumps(result))


if __name__ == "__main__":
    main()
