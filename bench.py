#!/usr/bin/env python
"""Long-range J benchmark on one MI355X.

One step = one long-range J build for one density (D(k) in HBM -> J(k) and E_J
in HBM): phase sum D(k) -> D(L), per-pair transforms, rho(G), V(G) and E_J, J
from V, back transform and J(L) -> J(k).  Workload: the 8-atom diamond-like
cell (a = 6.74 Bohr) with 10s6p3d uncontracted shells per atom on a 4x4x4
Gamma-centred k-mesh, omega 0.4, screening 1e-12, FP64.

`value` is J builds/s of the FP64 form, launched as the captured graph
(pwdf_build_j_graph) after an untimed autotune, from a region timed with
torch.cuda.synchronize() on both sides.  A second region of the same steps runs
with per-launch HIP events (library profiling mode: events on the stream each
kernel is launched on, launches serialised) and gives each kernel's average
duration for the roofline entry.  The same line reports the FP32-MFMA form and
16-density batches of both forms on the same workload, with their errors
(measured in a child process, so that a failure there is reported in
"extras_error" instead of ending the run), and the FP64 CPU oracle timed on the
host cores as the baseline.
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "long-range J builds/s + pair-G evals/s, FP32-MFMA vs FP64 at <=1e-7 Eh"
PEAK = {"fp64_valu_tflops": 78.6, "hbm_gbs": 8000.0}
CSRC = os.path.join(ROOT, "paper_2509_16460_amd", "csrc")
WORKLOAD = "diamond8_10s6p3d_k444_w0.4"


def kernel_source_hash():
    """Hash of every kernel and launch source: counter data older than this is stale."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(CSRC, f), "rb") as fh:
                h.update(f.encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


def flops_per_unit(name):
    """Algorithmic flops per work unit of the pair-G kernels.  The FP64 pair-G
    launches (rho_lo/hi, jpass_lo/hi) count their units in flops already: 8(L+1)+4
    per unique (pair, G of the half space, density) of class L in the factored
    form (an (L+1)-term complex multiply-add along the line plus the separable
    exponential/phase product).  The per-class FP32 launches count pair-G
    evaluations."""
    if name in ("rho_lo", "rho_hi", "jpass_lo", "jpass_hi"):
        return 1.0
    for pre in ("rho_mfma_L", "jpass_mfma_L"):
        if name.startswith(pre):
            L = int(name[len(pre):])
            return 8 * (L + 1) + 4
    return None


def bytes_per_unit(name):
    """Algorithmic HBM bytes per work unit of the phase kernels: one complex128
    value of J(k) written (phase_j, phase_j_heavy) or of D(k) read on the pair
    support (phase_d)."""
    return 16.0 if name in ("phase_j", "phase_j_heavy", "phase_d") else None


def roofline_entry(name, rec, traffic):
    avg_s = rec["ms"] / rec["launches"] * 1e-3
    units = rec["units"] / rec["launches"]
    fpu, bpu = flops_per_unit(name), bytes_per_unit(name)
    ent = {"kernel": name, "avg_launch_us": avg_s * 1e6, "units_per_launch": units}
    if bpu is not None:
        ach = units * bpu / avg_s / 1e9
        ent.update(bound="hbm", achieved=ach, peak=PEAK["hbm_gbs"], unit="GB/s", frac=ach / PEAK["hbm_gbs"],
                   traffic=traffic, bytes_per_unit=bpu, algorithmic_bytes_per_launch=units * bpu)
    elif fpu is not None:
        ach = units * fpu / avg_s / 1e12
        ent.update(bound="alu", achieved=ach, peak=PEAK["fp64_valu_tflops"], unit="TFLOP/s",
                   frac=ach / PEAK["fp64_valu_tflops"], traffic=traffic, flops_per_unit=fpu)
    else:
        ent.update(bound="alu", achieved=None, peak=None, unit=None, frac=None, traffic=traffic)
    return ent


def load_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary,
    or None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    ent = rec.get("kernels", {}).get(kernel)
    return None if not ent else ent.get("hbm_bytes_per_launch")


def cpu_baseline(prob, D, min_s=10.0, max_runs=8):
    from oracle import oracle as O
    cores = len(os.sched_getaffinity(0))
    runs, t0 = 0, time.perf_counter()
    ref = None
    while True:
        r = O.build_j(prob, D, want_rho=False, nthreads=cores)
        ref = ref or r
        runs += 1
        el = time.perf_counter() - t0
        if el >= min_s or runs >= max_runs:
            break
    return ({"value": runs / el, "unit": "J builds/s", "cores": cores, "kind": "oracle",
             "sample": f"{runs} full FP64 oracle J builds of the same workload, one density ({el:.1f} s)"}, ref)


def timed(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def extras(args):
    """FP32-MFMA form (one density) and 16-density batches of both forms on the
    same workload; prints one JSON object, writes the FP32 J(k) to --j32-out."""
    import numpy as np
    import torch
    from paper_2509_16460_amd import pwdf, synth

    torch.cuda.set_device(0)
    prob = synth.config_problem(2)
    D = synth.make_density(prob, 2000)
    Dt = torch.from_numpy(D[None]).cuda()
    ms = args.fp64_ms
    c32 = pwdf.LongRangeJ(prob, precision=pwdf.PWDF_FP32_MFMA, max_ndm=1)
    c32.autotune(1, None)
    J32 = torch.empty_like(Dt)
    E32 = torch.empty(1, dtype=torch.float64, device="cuda")
    ms32 = timed(torch, lambda: c32.build_j(Dt, J32, E32, graph=True), args.steps, args.warmup)
    fp32 = {"builds_per_s": 1e3 / ms32, "ms_per_build": ms32, "speedup_vs_fp64": ms / ms32,
            "E_J": float(E32.cpu()[0]), "seg_len": c32.stats()["seg_len"]}
    np.save(args.j32_out, J32.cpu().numpy()[0])
    del c32
    # 16-density batches (distinct densities), per-density throughput
    ndm = 16
    Db = torch.from_numpy(synth.make_densities(prob, ndm)).cuda()
    Jb = torch.empty_like(Db)
    Eb = torch.empty(ndm, dtype=torch.float64, device="cuda")
    batched = {}
    res = {}
    for name, prec in (("fp64", pwdf.PWDF_FP64), ("fp32_mfma", pwdf.PWDF_FP32_MFMA)):
        cb = pwdf.LongRangeJ(prob, precision=prec, max_ndm=ndm)
        cb.autotune(ndm, None)
        msb = timed(torch, lambda: cb.build_j(Db, Jb, Eb, graph=True), max(5, args.steps // 5), 2)
        res[name] = (Jb.clone(), Eb.clone())
        batched[name] = {"ndm": ndm, "ms_per_batch": msb, "density_builds_per_s": ndm * 1e3 / msb,
                         "speedup_vs_fp64_single": ndm * ms / msb}
        del cb
    batched["fp32_mfma"]["max_abs_dJ_vs_fp64_gpu"] = float((res["fp32_mfma"][0] - res["fp64"][0]).abs().max())
    batched["fp32_mfma"]["max_abs_dE_vs_fp64_gpu"] = float((res["fp32_mfma"][1] - res["fp64"][1]).abs().max())
    print(json.dumps({"fp32_mfma": fp32, "batched": batched}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the FP32-MFMA and batched measurements")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one plain device copy of this size (counter calibration)")
    ap.add_argument("--extras-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--fp64-ms", type=float, default=0.0, help=argparse.SUPPRESS)
    ap.add_argument("--j32-out", default="", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.extras_only:
        extras(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; runs on several GPUs are not "
                                   "supported (the long-range J build of one cell runs on one device)"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2509_16460_amd import pwdf, synth

    torch.cuda.set_device(0)
    prob = synth.config_problem(2)
    D = synth.make_density(prob, 2000)
    ctx = pwdf.LongRangeJ(prob, precision=pwdf.PWDF_FP64, max_ndm=1)
    ctx.autotune(1, None)
    st = ctx.stats()
    Dt = torch.from_numpy(D[None]).cuda()
    Jk = torch.empty_like(Dt)
    EJ = torch.empty(1, dtype=torch.float64, device="cuda")

    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # timed region: graph replay of the whole build
    ms = timed(torch, lambda: ctx.build_j(Dt, Jk, EJ, graph=True), args.steps, args.warmup)
    ms_eager = timed(torch, lambda: ctx.build_j(Dt, Jk, EJ), args.steps, 1)
    J64 = Jk.clone()
    E64 = float(EJ.cpu()[0])

    # profiled region: per-launch events, launches serialised on one stream
    ctx.profile_enable(True)
    for _ in range(args.steps):
        ctx.build_j(Dt, Jk, EJ)
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    dominant = max(prof, key=lambda k: prof[k]["ms"] / prof[k]["launches"])
    roof = roofline_entry(dominant, prof[dominant], load_traffic(dominant))
    tot = sum(x["ms"] for x in prof.values())
    kernels = {k: {"launches": v["launches"], "avg_us": v["ms"] / v["launches"] * 1e3, "share": v["ms"] / tot}
               for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])}
    second = [roofline_entry(k, prof[k], load_traffic(k)) for k in kernels
              if k != dominant and (flops_per_unit(k) or bytes_per_unit(k))][:4]

    builds_per_s = 1e3 / ms
    pairG = st["pairG_evals"]
    out = {
        "metric": METRIC,
        "value": builds_per_s,
        "unit": "J builds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "atoms": prob.natm, "nbf": prob.nbf, "nk": prob.nk,
                   "omega": prob.omega, "nG": st["nG"], "unique_pairs": st["npairs"], "ndm": 1,
                   "precision": "fp64", "launch": "graph replay, autotuned", "seg_len": st["seg_len"]},
        "pair_G_evals_per_s": pairG * builds_per_s,
        "pair_G_evals_per_build": pairG,
        "ms_per_step_eager": ms_eager,
        "roofline": roof,
        "roofline_next": second,
        "kernels": kernels,
        "E_J": E64,
    }

    J32 = None
    if not args.no_extras:
        # FP32-MFMA form and 16-density batches in a child process (one more GPU
        # process for the duration): a failure there is reported, not fatal
        print("bench: FP32-MFMA and batched measurements (child process)", file=sys.stderr, flush=True)
        with tempfile.TemporaryDirectory() as td:
            j32p = os.path.join(td, "j32.npy")
            cmd = [sys.executable, os.path.abspath(__file__), "--extras-only", "--steps", str(args.steps),
                   "--warmup", str(args.warmup), "--fp64-ms", repr(ms), "--j32-out", j32p]
            try:
                r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
                lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
                if r.returncode == 0 and lines:
                    out.update(json.loads(lines[-1]))
                    J32 = np.load(j32p)
                else:
                    out["extras_error"] = f"exit status {r.returncode}: {r.stderr[-400:]}"
            except subprocess.TimeoutExpired:
                out["extras_error"] = "timed out after 900 s"
        print("bench: extras done", file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        base, ref = cpu_baseline(prob, D)
        out["cpu_baseline"] = base
        out["parity_vs_oracle"] = {"dE_J": abs(E64 - ref["E_G"]),
                                   "max_abs_dJ": float(np.max(np.abs(J64.cpu().numpy()[0] - ref["J"])))}
        if "fp32_mfma" in out and J32 is not None:
            out["fp32_mfma"]["dE_J_vs_oracle"] = abs(out["fp32_mfma"]["E_J"] - ref["E_G"])
            out["fp32_mfma"]["max_abs_dJ_vs_oracle"] = float(np.max(np.abs(J32 - ref["J"])))
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out))


if __name__ == "__main__":
    main()
