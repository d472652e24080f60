#!/usr/bin/env python
"""Long-range J benchmark on one MI355X.

One step = one batched long-range J build of 16 densities on the rock-salt
slab (32 atoms, a = 7.96 Bohr, 2x2 surface cell, 4 layers, 20 Bohr vacuum;
8s5p3d1f uncontracted shells per element; 6x6x1 Gamma-centred k-mesh;
omega 0.4, screening 1e-12 with per-pair G cuts): D(k) of every density in
HBM -> J(k) and E_J in HBM, i.e. the phase sum D(k) -> D(L), per-pair
transforms, rho(G), V(G) and E_J, J from V, back transform and J(L) -> J(k).
The headline form is the FP32-MFMA one (pair-G tiles in FP32 on the matrix
cores, the head of the G set in FP64 tiles on FP64 MFMA; phase sums,
transforms and energies in FP64), launched as the captured graph after an
untimed autotune, with D(k) read and J(k) written on the pair support only,
packed (the layouts PWDF_DK_PACKED and PWDF_JK_PACKED: [density][k][support
element]; the dense D(k) is gathered into that layout before the timed
region).  `value` is density J builds/s (16 per step) from a region timed with
torch.cuda.synchronize() on both sides; the same build reading the dense
[density][k][nbf][nbf] D(k) is timed before it ("dense_dk_input").

Beside it, on the same slab and densities: the FP64 form with one density per
call (the plain form; the ratio of the two is the batched-FP32 speedup) and
with 16 per call, the FP32-MFMA batch without per-pair cuts, the errors
against each other and against the FP64 oracle; then (child process, so that a
failure there is reported in "extras_error" instead of ending the run) the FP64
form on the monoclinic molecular crystal and on the diamond-like cell, and the
compact/diffuse classification on a cell with diffuse shells (the diffuse pairs
by their analytic transforms and by GPW).  A
second, profiled region of the headline form brackets every launch with HIP
events on its stream and gives each kernel's average duration for the roofline
entry.  The FP64 CPU oracle, timed on the host cores for one slab density, is
the baseline.
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
PEAK = {"fp64_valu_tflops": 78.6, "fp64_mfma_tflops": 78.6, "fp32_mfma_tflops": 157.3, "hbm_gbs": 8000.0}
CSRC = os.path.join(ROOT, "paper_2509_16460_amd", "csrc")
WORKLOAD = "rocksalt_slab32_8s5p3d1f_k661_w0.4_ndm16_paircut"
NDM = 16


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
    """Algorithmic flops per work unit of the pair-G kernels: 8(L+1)+4 per unique
    (pair, G of the half space, density) of class L in the factored form (an
    (L+1)-term complex multiply-add along the G line plus the separable
    exponential/phase product).  The FP64 launches rho_lo/hi and jpass_lo/hi
    count their units in these flops already; the per-class MFMA launches (FP32
    tiles, and FP64 tiles of the head of the G set) count pair-G evaluations.  The
    density transform and the back transform count their algorithmic flops (two
    per term of the E-coefficient contraction and per Hermite -> monomial table
    entry, per pair and density) on the FP64 VALU."""
    if name in ("rho_lo", "rho_hi", "jpass_lo", "jpass_hi", "transform", "back"):
        return 1.0
    for pre in ("rho_mfma_L", "jpass_mfma_L", "rho_head_L", "jpass_head_L"):
        if name.startswith(pre):
            L = int(name[len(pre):])
            return 8 * (L + 1) + 4
    return None


def bytes_per_unit(name):
    """Algorithmic HBM bytes per work unit of the phase kernels: one complex128
    value of J(k) written (phase_j) or of D(k) read (phase_d) on the pair support."""
    return 16.0 if name in ("phase_j", "phase_d") else None


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
        mfma = "mfma" in name or "head" in name
        peak = PEAK["fp32_mfma_tflops"] if "mfma" in name else (
            PEAK["fp64_mfma_tflops"] if "head" in name else PEAK["fp64_valu_tflops"])
        ach = units * fpu / avg_s / 1e12
        ent.update(bound="mfma" if mfma else "alu", achieved=ach, peak=peak, unit="TFLOP/s", frac=ach / peak,
                   traffic=traffic, flops_per_unit=fpu, algorithmic_flops_per_launch=units * fpu)
    else:
        ent.update(bound="alu", achieved=None, peak=None, unit=None, frac=None, traffic=traffic)
    return ent


def load_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` on `workload` from the committed rocprofv3
    counter summary, or None when the kernel sources changed since."""
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
    ent = rec.get("workloads", {}).get(workload, {}).get(kernel)
    return None if not ent else ent.get("hbm_bytes_per_launch")


def timed(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def profile_kernels(torch, ctx, fn, steps):
    """Per-kernel launch statistics from the library's event profiling (events on
    the stream each kernel runs on, launches serialised)."""
    ctx.profile_enable(True)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    return prof


def kernel_table(prof):
    tot = sum(x["ms"] for x in prof.values())
    return {k: {"launches": v["launches"], "avg_us": v["ms"] / v["launches"] * 1e3, "share": v["ms"] / tot}
            for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])}


def single_fp64(torch, pwdf, prob, Dt, steps, warmup):
    """FP64 form, one density per call, packed D(k) and J(k), graph replay, autotuned."""
    ctx = pwdf.LongRangeJ(prob, precision=pwdf.PWDF_FP64, max_ndm=1)
    ctx.set_jk_layout(pwdf.PWDF_JK_PACKED)
    ctx.set_dk_layout(pwdf.PWDF_DK_PACKED)
    Dt = ctx.pack_dk(Dt)
    ctx.autotune(1, None)
    J = torch.empty((1, prob.nk, ctx.stats()["jk_support"]), dtype=Dt.dtype, device=Dt.device)
    E = torch.empty(1, dtype=torch.float64, device="cuda")
    ms = timed(torch, lambda: ctx.build_j(Dt, J, E, graph=True), steps, warmup)
    st = ctx.stats()
    prof = profile_kernels(torch, ctx, lambda: ctx.build_j(Dt, J, E), max(3, steps // 4))
    return ctx, J, E, ms, st, prof


def extras(args):
    """FP64 single-density builds of the molecular crystal and the diamond-like
    cell, and of a cell with diffuse shells under the compact/diffuse
    classification (the DD pairs by their analytic transforms and by GPW);
    prints one JSON object."""
    import torch
    from paper_2509_16460_amd import pwdf, synth

    torch.cuda.set_device(0)
    out = {}
    for cfg, name in ((5, "molecular_crystal48_k333_w0.5_fp64_paircut"), (2, "diamond8_k444_w0.4_fp64_paircut")):
        print(f"bench: extras {name}: autotune + timed region", file=sys.stderr, flush=True)
        prob = synth.config_problem(cfg).with_(pair_gcut=1)
        D = synth.make_density(prob, 1000 * cfg)
        Dt = torch.from_numpy(D[None]).cuda()
        ctx, J, E, ms, st, prof = single_fp64(torch, pwdf, prob, Dt, args.steps, args.warmup)
        kt = kernel_table(prof)
        out[name] = {"builds_per_s": 1e3 / ms, "ms_per_build": ms, "pair_G_evals_per_s": st["pairG_evals"] * 1e3 / ms,
                     "nG": st["nG"], "unique_pairs": st["npairs"], "nbf": st["nbf"], "nk": st["nk"],
                     "seg_len": st["seg_len"], "E_J": float(E.cpu()[0]),
                     "roofline": [roofline_entry(k, prof[k], None) for k in list(kt)[:4]]}
        del ctx, J, E, Dt
        torch.cuda.empty_cache()
        print(f"bench: extras {name} {ms:.3f} ms", file=sys.stderr, flush=True)
    # compact/diffuse classification on a cell with diffuse shells: the DD pairs by
    # their analytic transforms and by GPW (real-space grid), FP64, one density
    prob = synth.diffuse_problem(a=11.0, natm=2)
    D = synth.make_density(prob, 7000)
    Dt = torch.from_numpy(D[None]).cuda()
    res, Js = {}, {}
    for route in (0, 1):
        pr = prob.with_(dd_gpw=route)
        print(f"bench: extras classification, {'GPW' if route else 'analytic'} route", file=sys.stderr, flush=True)
        # default launch shapes (no autotune), graph replay
        ctx = pwdf.LongRangeJ(pr, precision=pwdf.PWDF_FP64, max_ndm=1)
        ctx.set_jk_layout(pwdf.PWDF_JK_PACKED)
        ctx.set_dk_layout(pwdf.PWDF_DK_PACKED)
        Dp = ctx.pack_dk(Dt)
        J = torch.empty((1, pr.nk, ctx.stats()["jk_support"]), dtype=Dt.dtype, device=Dt.device)
        E = torch.empty(1, dtype=torch.float64, device="cuda")
        ms = timed(torch, lambda: ctx.build_j(Dp, J, E, graph=True), min(args.steps, 10), 2)
        st = ctx.stats()
        prof = profile_kernels(torch, ctx, lambda: ctx.build_j(Dp, J, E), 3)
        kt = kernel_table(prof)
        dd = {k: v["avg_us"] for k, v in kt.items() if k in ("rho_dd", "jpass_dd", "combine_dd", "gpw_rho", "gpw_j",
                                                              "gpw_add")}
        res["gpw" if route else "analytic"] = {"ms_per_build": ms, "builds_per_s": 1e3 / ms, "dd_kernels_us": dd,
                                               "E_J": float(E.cpu()[0]), "gpw_grid": list(st["gpw_grid"])}
        Js[route] = J.clone()
        del ctx, J, E
        torch.cuda.empty_cache()
    res["workload"] = prob.name + "_k222_w0.5_fp64_cd (default launch shapes)"
    res.update(natm=prob.natm, nbf=prob.nbf, nk=prob.nk, unique_pairs=st["npairs"], dd_pairs=st["npairs_dd"],
               nG=st["nG"], max_abs_dJ_gpw_vs_analytic=float((Js[0] - Js[1]).abs().max()))
    out["classification"] = res
    print(f"bench: extras classification {res['analytic']['ms_per_build']:.3f} / {res['gpw']['ms_per_build']:.3f} ms",
          file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


def rocprof_summary(paths, last):
    """Markdown table per kernel of rocprofv3 CSV output, over the last `last`
    dispatches of each kernel (0: all; the timed and profiled regions of a run
    come after its autotune): from *_kernel_trace.csv the dispatch count and
    average duration in us; from *_counter_collection.csv the average of every
    counter per dispatch (FETCH_SIZE / WRITE_SIZE in KiB, as rocprofv3 reports
    them)."""
    import csv
    import re
    disp = {}
    for path in paths:
        with open(path) as fh:
            for r in csv.DictReader(fh):
                name = r.get("Kernel_Name") or ""
                m = re.search(r"pwdf::(k_\w+)(<[^>]*>)?", name)
                key = (m.group(1) + (m.group(2) or "")) if m else name[:48]
                dd = disp.setdefault(key, {})
                e = dd.setdefault(int(r["Dispatch_Id"]), {})
                e["dur_us"] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
                if "Counter_Name" in r:
                    e[r["Counter_Name"]] = e.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    rows = {}
    for key, dd in disp.items():
        ids = sorted(dd)[-last:] if last else sorted(dd)
        cols = {c for i in ids for c in dd[i]}
        rows[key] = {"dispatches": len(ids)}
        for c in cols:
            vals = [dd[i][c] for i in ids if c in dd[i]]
            rows[key][c] = sum(vals) / len(vals)
    cols = ["dispatches", "dur_us"] + sorted({c for d in rows.values() for c in d} - {"dispatches", "dur_us"})
    print("| kernel | " + " | ".join(cols) + " |")
    print("|---" * (len(cols) + 1) + "|")
    for k in sorted(rows, key=lambda k: -rows[k]["dur_us"] * rows[k]["dispatches"]):
        print(f"| `{k}` | " + " | ".join(f"{rows[k][c]:.4g}" if c in rows[k] else "" for c in cols) + " |")


def profile_name(kernel):
    """The bench's profile name (pwdf_profile_*) of a device kernel, or None."""
    import re
    m = re.search(r"pwdf::(k_\w+)(?:<(\d+)[^>]*>)?", kernel)
    if not m:
        return None
    k, L = m.group(1), m.group(2)
    fixed = {"k_phase_j_all": "phase_j", "k_phase_d": "phase_d", "k_back_all": "back", "k_back_30": "back",
             "k_transform_all": "transform", "k_ysum": "back", "k_reduce_rows": "reduce", "k_reduce": "reduce", "k_fold_j": "fold_j",
             "k_wprep": "wprep"}
    if k in fixed:
        return fixed[k]
    per_class = {"k_rho_mfma": "rho_mfma_L", "k_rho_head": "rho_head_L", "k_jpass_mfma": "jpass_mfma_L",
                 "k_jpass_head": "jpass_head_L"}
    return per_class[k] + L if k in per_class and L is not None else None


def traffic_json(fetch_csv, write_csv, last):
    """profiles/traffic_counters.json from two rocprofv3 counter runs of the
    headline leg (FETCH_SIZE, then WRITE_SIZE, both with --calib-copy-mib): each
    counter scaled by what it reads for the calibration kernel (torch's neg over
    the given size, reading and writing it once), HBM bytes per launch of each
    profile kernel = the sum over its device kernels of their average over the
    last `last` dispatches."""
    import csv
    per = {}
    calib = {}
    for path, counter in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        disp = {}
        neg = 0.0
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") != counter:
                    continue
                name, v = r["Kernel_Name"], float(r["Counter_Value"])
                if "neg_kernel" in name:
                    neg = max(neg, v)
                disp.setdefault(name, {})[int(r["Dispatch_Id"])] = v
        calib[counter] = neg
        for name, dd in disp.items():
            pn = profile_name(name)
            if pn is None:
                continue
            ids = sorted(dd)[-last:]
            per.setdefault(pn, {}).setdefault(counter, 0.0)
            per[pn][counter] += sum(dd[i] for i in ids) / len(ids)
    if not calib.get("FETCH_SIZE") or not calib.get("WRITE_SIZE"):
        raise SystemExit("no calibration kernel found (run the counter passes with --calib-copy-mib)")
    # the calibration kernel moves the size once each way; KiB per dispatch
    size_kib = max(calib["WRITE_SIZE"], calib["FETCH_SIZE"])
    f_fetch, f_write = size_kib / calib["FETCH_SIZE"], size_kib / calib["WRITE_SIZE"]
    out = {"source_hash": kernel_source_hash(), "workloads": {WORKLOAD: {}},
           "calibration": {"fetch_factor": f_fetch, "write_factor": f_write, "calib_kib": size_kib},
           "note": "HBM bytes per launch = (FETCH_SIZE x fetch_factor + WRITE_SIZE x write_factor) KiB x 1024, "
                   f"average of the last {last} dispatches of each device kernel, summed per profile kernel"}
    for pn, c in sorted(per.items()):
        out["workloads"][WORKLOAD][pn] = {
            "fetch_kib_raw": c.get("FETCH_SIZE", 0.0), "write_kib_raw": c.get("WRITE_SIZE", 0.0),
            "hbm_bytes_per_launch": 1024.0 * (c.get("FETCH_SIZE", 0.0) * f_fetch + c.get("WRITE_SIZE", 0.0) * f_write)}
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"wrote {path}: fetch x{f_fetch:.4f}, write x{f_write:.4f}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the molecular crystal and diamond cell")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one plain streaming kernel over this size (counter calibration)")
    ap.add_argument("--extras-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--only-headline", action="store_true",
                    help="run the headline FP32-MFMA batch only (autotune, timed and profiled regions): the "
                         "command the rocprofv3 summaries under profiles/ are taken with")
    ap.add_argument("--rocprof-summary", nargs="+", metavar="CSV",
                    help="print a per-kernel summary of rocprofv3 CSV output (kernel_trace or "
                         "counter_collection files) instead of benchmarking")
    ap.add_argument("--last", type=int, default=0, help="with --rocprof-summary: the last N dispatches per kernel")
    ap.add_argument("--tune-cache", default=None,
                    help="tune cache file of the headline's autotune (a profiling run can reuse the launch shapes "
                         "an earlier run chose instead of timing candidates under the profiler)")
    ap.add_argument("--traffic-json", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic_counters.json from the two counter runs (with --last N)")
    args = ap.parse_args()
    if args.traffic_json:
        traffic_json(args.traffic_json[0], args.traffic_json[1], args.last or 3)
        return
    if args.rocprof_summary:
        rocprof_summary(args.rocprof_summary, args.last)
        return
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
    log = lambda m: print("bench: " + m, file=sys.stderr, flush=True)  # noqa: E731
    prob = synth.config_problem(4).with_(pair_gcut=1)
    log("slab overlap for the density scale")
    Sk = synth.overlap_k(prob)
    Db = synth.make_densities_torch(prob, NDM, 1000 * prob.seed, Sk)
    del Sk
    Eb = torch.empty(NDM, dtype=torch.float64, device="cuda")

    if args.calib_copy_mib > 0:
        # a plain streaming kernel of known traffic (reads and writes the size
        # given once each; torch's neg kernel, found by name in the counter
        # output), for the scale of the FETCH_SIZE / WRITE_SIZE counters
        n = args.calib_copy_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.neg(a, out=b)
        torch.cuda.synchronize()
        del a, b

    # headline: FP32-MFMA form, 16 densities per call, graph replay
    log("FP32-MFMA batch: autotune")
    c32 = pwdf.LongRangeJ(prob, precision=pwdf.PWDF_FP32_MFMA, max_ndm=NDM)
    c32.set_jk_layout(pwdf.PWDF_JK_PACKED)
    c32.set_dk_layout(pwdf.PWDF_DK_PACKED)
    c32.autotune(NDM, args.tune_cache)
    st = c32.stats()
    mu, nu = c32.jk_support()
    Jb = torch.empty((NDM, prob.nk, st["jk_support"]), dtype=Db.dtype, device="cuda")
    # the same build reading the dense D(k), timed first so that the last launches
    # of every kernel (those the profiles average) are the packed form's
    c32.set_dk_layout(pwdf.PWDF_DK_FULL)
    log("FP32-MFMA batch, dense D(k): timed region")
    ms_dense = timed(torch, lambda: c32.build_j(Db, Jb, Eb, graph=True), args.steps, args.warmup)
    Jd0 = Jb[0].clone()
    dense_dk = {"ms_per_step": ms_dense, "builds_per_s": NDM * 1e3 / ms_dense,
                "dk_support_elements": c32.stats()["dk_support"]}
    c32.check_input()
    c32.set_dk_layout(pwdf.PWDF_DK_PACKED)
    Dp = c32.pack_dk(Db)  # outside the timed region: the density as the caller holds it
    log("FP32-MFMA batch: timed region")
    ms = timed(torch, lambda: c32.build_j(Dp, Jb, Eb, graph=True), args.steps, args.warmup)
    J32_0 = Jb[0].clone()
    E32 = Eb.cpu().numpy().copy()
    prof = profile_kernels(torch, c32, lambda: c32.build_j(Dp, Jb, Eb), max(3, args.steps // 4))
    c32.check_input()
    dense_dk["max_abs_dJ_vs_packed"] = float((Jd0 - J32_0).abs().max())
    del Dp, Jd0
    dominant = max(prof, key=lambda k: prof[k]["ms"] / prof[k]["launches"])
    roof = roofline_entry(dominant, prof[dominant], load_traffic(WORKLOAD, dominant))
    kernels = kernel_table(prof)
    second = [roofline_entry(k, prof[k], load_traffic(WORKLOAD, k)) for k in kernels
              if k != dominant and (flops_per_unit(k) or bytes_per_unit(k))][:5]
    del c32
    torch.cuda.empty_cache()

    if args.only_headline:
        print(json.dumps({"metric": METRIC, "value": NDM * 1e3 / ms, "unit": "J builds/s", "ms_per_step": ms,
                          "config": {"workload": WORKLOAD}, "roofline": roof, "kernels": kernels,
                          "dense_dk_input": dense_dk}), flush=True)
        return

    # side legs: the FP32-MFMA batch without per-pair cuts, the FP64 form with 16
    # densities per call (no autotune, graph replay)
    def side(pr, prec):
        c = pwdf.LongRangeJ(pr, precision=prec, max_ndm=NDM)
        c.set_jk_layout(pwdf.PWDF_JK_PACKED)
        c.set_dk_layout(pwdf.PWDF_DK_PACKED)
        Dq = c.pack_dk(Db)
        J = torch.empty((NDM, pr.nk, c.stats()["jk_support"]), dtype=Db.dtype, device="cuda")
        E = torch.empty(NDM, dtype=torch.float64, device="cuda")
        t = timed(torch, lambda: c.build_j(Dq, J, E, graph=True), max(5, args.steps // 2), args.warmup)
        del Dq
        r = {"ms_per_step": t, "builds_per_s": NDM * 1e3 / t, "pair_G_evals_per_density_build": c.stats()["pairG_evals"]}
        del c, J, E
        torch.cuda.empty_cache()
        return r
    log("side legs: FP32-MFMA batch without cuts, FP64 batch")
    nocut32 = side(prob.with_(pair_gcut=0), pwdf.PWDF_FP32_MFMA)
    batch64 = side(prob, pwdf.PWDF_FP64)

    # the plain form on the same slab: FP64, one density per call
    log("FP64 single density: autotune + timed region")
    D0 = Db[0:1]
    c64, J64, E64t, ms64, st64, prof64 = single_fp64(torch, pwdf, prob, D0, args.steps, args.warmup)
    E64 = float(E64t.cpu()[0])
    dJ_32_64 = float((J32_0 - J64[0]).abs().max())
    del c64
    torch.cuda.empty_cache()

    dens_per_s = NDM * 1e3 / ms
    out = {
        "metric": METRIC,
        "value": dens_per_s,
        "unit": "J builds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "atoms": prob.natm, "nbf": prob.nbf, "nk": prob.nk, "omega": prob.omega,
                   "nG": st["nG"], "unique_pairs": st["npairs"], "ndm_per_step": NDM,
                   "precision": "fp32_mfma (pair-G tiles FP32 on MFMA, head of the G set (v(G) >= 2^-20 max v) FP64 on MFMA; phase "
                                "sums, transforms, energy FP64)",
                   "screening": "eps 1e-12, per-pair G cuts", "nG_head": st["nG_head"],
                   "jk_layout": "packed support", "jk_support_elements": st["jk_support"],
                   "dk_layout": "packed support", "dk_support_elements_read": st["dk_support"],
                   "launch": "graph replay, autotuned", "seg_len": st["seg_len"]},
        "pair_G_evals_per_s": st["pairG_evals"] * dens_per_s,
        "pair_G_evals_per_density_build": st["pairG_evals"],
        "pair_G_fp64_head_fraction": st["pairG_head"] / max(1.0, st["pairG_evals"]),
        "dense_dk_input": dense_dk,
        "fp32_batch_without_pair_cuts": nocut32,
        "fp64_batch16": batch64,
        "roofline": roof,
        "roofline_next": second,
        "kernels": kernels,
        "fp64_single": {"builds_per_s": 1e3 / ms64, "ms_per_build": ms64,
                        "pair_G_evals_per_s": st64["pairG_evals"] * 1e3 / ms64, "seg_len": st64["seg_len"],
                        "kernels": kernel_table(prof64)},
        "fp32_batch_speedup_vs_fp64_single": (ms64 * NDM) / ms,
        "fp32_vs_fp64": {"density": 0, "dE_J": abs(float(E32[0]) - E64), "max_abs_dJ": dJ_32_64},
        "E_J": [float(x) for x in E32],
    }

    if not args.no_extras:
        log("molecular crystal and diamond cell (child process)")
        cmd = [sys.executable, os.path.abspath(__file__), "--extras-only", "--steps", str(args.steps),
               "--warmup", str(args.warmup)]
        try:
            # the child's progress lines go straight to this process's stderr
            r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, timeout=600)
            lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
            if r.returncode == 0 and lines:
                out["other_workloads"] = json.loads(lines[-1])
            else:
                out["extras_error"] = f"exit status {r.returncode}"
        except subprocess.TimeoutExpired:
            out["extras_error"] = "timed out after 600 s"

    if not args.no_cpu_baseline:
        from oracle import oracle as O
        log("oracle on one slab density (CPU baseline)")
        cores = len(os.sched_getaffinity(0))
        Dh = Db[0].cpu().numpy()
        t0 = time.perf_counter()
        ref = O.build_j(prob, Dh, want_rho=False, nthreads=cores)
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 1.0 / el, "unit": "J builds/s", "cores": cores, "kind": "oracle",
                               "sample": f"one full FP64 oracle J build of slab density 0 ({el:.1f} s); "
                                         f"the batch of {NDM} would take {NDM * el:.0f} s"}
        Jr = ref["J"][:, mu, nu]  # the packed element order
        out["parity_vs_oracle"] = {
            "fp64_single": {"dE_J": abs(E64 - ref["E_G"]),
                            "max_abs_dJ": float(np.max(np.abs(J64[0].cpu().numpy() - Jr)))},
            "fp32_mfma_batch_density0": {"dE_J": abs(float(E32[0]) - ref["E_G"]),
                                         "max_abs_dJ": float(np.max(np.abs(J32_0.cpu().numpy() - Jr)))},
            "max_abs_J": float(np.max(np.abs(Jr))), "E_J": ref["E_G"]}
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
