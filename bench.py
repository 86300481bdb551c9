"""Benchmark of the coupled FFT solve on one MI355X.

A step is one load increment of the 256^3 short-fibre composite (991 planar-
isotropic E-glass fibres, aspect ratio 20, 20 % volume fraction, PA66 matrix)
solved by Newton-CG with FP32 fields and FP64 reductions / return mapping:
per-voxel constitutive update, 3D FFT, Green operator, inverse FFT and the
Krylov update, for the mechanical and the conduction fields. The value is
mechanical voxel-iterations per second (one voxel-iteration = one
application of the FFT pipeline to one voxel), with the inputs resident in
HBM. Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "voxel-iters/s coupled FFT solve; surrogate vs FFT Gauss-pts/s at 1e-3 err"
HBM_PEAK_GBS = 8000.0
# sources whose change makes stored counter data stale (kernels and launch shapes)
KERNEL_SOURCES = ("paper_2109_14403_amd/csrc/pipeline.h", "paper_2109_14403_amd/csrc/fft_core.h",
                  "paper_2109_14403_amd/csrc/pa66.h",
                  "paper_2109_14403_amd/csrc/pointwise.hip", "paper_2109_14403_amd/csrc/pointwise.h",
                  "paper_2109_14403_amd/csrc/common.h", "paper_2109_14403_amd/csrc/pipe_inst.hip",
                  "paper_2109_14403_amd/csrc/pipe_launch.h")


CALIB_FLOATS = 1 << 28
NETWORK_PARAMS_MACS = 32 * 256 + 3 * 256 * 256 + 256 * 10   # multiply-adds per row of one network
PMC_KINDS = {"xfwd": "k_xfwd", "ypass": "k_ypass", "zgreen": "k_zgreen", "xinv": "k_xinv", "eval": "k_eval",
             "commit": "k_commit_vox", "history": "k_history", "init": "k_init"}


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(kind, n, fp_bytes, matrix_fraction):
    """Minimum bytes one launch of a mechanical kernel moves on one n^3 problem,
    as (residual evaluation, first CG iteration of a Newton step, later CG
    iteration). Spectra hold n * n * (n/2 + 1) * 6 complex values; the
    direction field of plastic voxels is not counted (a lower bound)."""
    v = float(n) ** 3
    spec = n * n * (n // 2 + 1) * 6 * 2 * fp_bytes
    field = 6 * fp_bytes * v
    if kind in ("yfwd", "yinv", "zgreen"):
        return 2 * spec, 2 * spec, 2 * spec
    if kind == "xfwd":
        # eval: read stress, write spectra. CG: read r (+ p, x), tangent factors
        # and phase, write p (+ x) and spectra
        tang = 2 * fp_bytes * v + v
        return field + spec, 2 * field + tang + spec, 5 * field + tang + spec
    if kind == "xinv":   # eval: read spectra and stress, write r; CG: read spectra and r, write r
        return spec + 2 * field, spec + 2 * field, spec + 2 * field
    if kind == "eval":   # read strain, phase, PA66 eps_p, eps_vp and history sums; write stress, tangent factors
        return 2 * field + v + matrix_fraction * v * 14 * 8 + 2 * fp_bytes * v, 0.0, 0.0
    return None


def solve_bytes(n, fp_bytes, matrix_fraction, n_state, n_eval, n_cg, n_first, increments, thermal):
    """Algorithmic bytes of every kernel of `increments` timed increments, per
    kernel (GB): the mechanical pipeline launches (n_eval residual
    evaluations, n_first first and n_cg - n_first later CG iterations), the
    per-increment kernels (init, branch history sums, commit) and the
    conduction solve (`thermal`: its launches of each pass kernel, counted at
    the residual-evaluation size, a lower bound). Evaluation launches of CG
    iterations return at once and move nothing; reductions are left out
    (kilobytes)."""
    v = float(n) ** 3
    mv = matrix_fraction * v
    field = 6 * fp_bytes * v
    launches = n_eval + n_cg
    xf = algorithmic_bytes("xfwd", n, fp_bytes, matrix_fraction)
    ev = algorithmic_bytes("eval", n, fp_bytes, matrix_fraction)[0]
    out = {
        "xfwd": n_eval * xf[0] + n_first * xf[1] + (n_cg - n_first) * xf[2],
        "ypass": 2 * launches * algorithmic_bytes("yfwd", n, fp_bytes, matrix_fraction)[0],
        "zgreen": launches * algorithmic_bytes("zgreen", n, fp_bytes, matrix_fraction)[0],
        "xinv": launches * algorithmic_bytes("xinv", n, fp_bytes, matrix_fraction)[0],
        # every evaluation after an increment's first applies the last CG step
        # x += alpha p first: read p, write x
        "eval": n_eval * ev + (n_eval - increments) * 2 * field,
        # x = x^n + dE: read x^n, write x
        "init": increments * 2 * field,
        # read the viscous strains of the branches, write 8 FP64 slots (the
        # PA66 voxels' compacted arrays: no phase test)
        "history": increments * (mv * ((n_state - 7) * 8 + 8 * 8)),
        # read x, x^n, phase, the state and the history sums; write the state, x^n, the stress
        "commit": increments * (4 * field + v + mv * (2 * n_state * 8 + 8 * 8)),
    }
    spec3 = n * n * (n // 2 + 1) * 3 * 2 * fp_bytes
    f3 = 3 * fp_bytes * v
    th = (thermal.get("xfwd", 0) * (f3 + spec3) + thermal.get("yfwd", 0) * 2 * spec3
          + thermal.get("yinv", 0) * 2 * spec3 + thermal.get("zgreen", 0) * 2 * spec3
          + thermal.get("xinv", 0) * (spec3 + 2 * f3) + thermal.get("init", 0) * 2 * f3
          + thermal.get("commit", 0) * (f3 + v))
    out["conduction"] = th
    return {k: val / 1e9 for k, val in out.items()}


def _host_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "cpu_model": model}


def counter_solve_bytes(n, n_eval, n_cg, increments):
    """HBM GB that the counters measured, for the timed increments: bytes per
    working launch of each mechanical kernel (profiles/<kind>_fibres<n>_pmc.json,
    current kernel sources only) times its working launches (n_eval residual
    evaluations, n_cg CG iterations; the evaluation launches of CG iterations
    return at once). None if one is missing."""
    it = n_eval + n_cg
    launches = {"xfwd": it, "ypass": 2 * it, "zgreen": it, "xinv": it, "eval": n_eval, "commit": increments,
                "history": increments, "init": increments}
    h = kernel_source_hash()
    tot = 0.0
    for kind, nl in launches.items():
        path = os.path.join(ROOT, "profiles", f"{kind}_fibres{n}_pmc.json")
        if not os.path.exists(path):
            return None
        pm = json.load(open(path))
        if pm.get("source_hash") != h:
            return None
        tot += pm["bytes_per_launch"] * nl
    return tot / 1e9


def cpu_baseline(phases, laws, reps=2):
    """The oracle as it stands, timed on this host's cores (its library FFT on
    every core, and on one thread): CG operator applications A p = P[C p] on
    the full 256^3 grid (the bench workload); the whole 10-increment history of
    the 16^3 sphere (basic scheme, FP64, tol 1e-8); and the first Newton-CG
    increment of the 64^3 sphere composite with its PA66 return map (tol 1e-6)."""
    from oracle import fourier, solver
    from paper_2109_14403_amd import workloads as W

    host = _host_info()
    cores = host["nproc"]
    cell = solver.Cell(phases, laws)
    rng = np.random.default_rng(0)
    shape = phases.shape
    tan = np.zeros((6, 6) + shape)
    for i, law in enumerate(cell.laws):
        if law.inelastic:
            mats = law.branch_matrices(313.15, 0.8)
            C = law.Cinf.copy()
            for j, (B, M) in enumerate(mats):
                C = C + law.C_i[j] @ (np.eye(6) - M)
        else:
            C = law.C
        tan[:, :, cell.masks[i]] = C[:, :, None]

    def operator_rate(workers):
        fourier.WORKERS = workers
        p = rng.normal(size=(6,) + shape)
        t0 = time.perf_counter()
        for _ in range(reps):
            ap = cell.project(np.einsum("ab...,b...->a...", tan, p))
            _ = float((p * ap).sum())
            p = ap
        return reps * float(np.prod(shape)) / (time.perf_counter() - t0)

    try:
        rate_all = operator_rate(cores)
        rate_one = operator_rate(1)
        fourier.WORKERS = cores
        wl = W.small_sphere_workload()
        ref = solver.Cell(wl.phases, wl.laws)
        t0 = time.perf_counter()
        its = 0
        for st in wl.history:
            o = ref.solve_increment(st.strain, st.theta, st.grad, st.dt, scheme="basic", tol=1e-8)
            its += o["iterations"]
        t1 = time.perf_counter() - t0
        wl2 = W.sphere_composite_workload(64, seed=2)
        ref2 = solver.Cell(wl2.phases, wl2.laws)
        st = wl2.history[0]
        t0 = time.perf_counter()
        o2 = ref2.solve_increment(st.strain, st.theta, st.grad, st.dt, tol=1e-6)
        t2 = time.perf_counter() - t0
    finally:
        fourier.WORKERS = 1
    pipes2 = o2["iterations"] + o2["krylov"]
    return {"value": rate_all, "unit": "voxel-iters/s", "cores": cores, "kind": "oracle",
            "sample": f"{reps} CG operator applications (tangent, FFT, projector, inverse FFT) of the FP64 "
                      "oracle on the full 256^3 grid",
            "single_thread_value": rate_one, "host": host,
            "config1_history": {"workload": "sphere16 thermoelastic, basic scheme, 10 increments", "seconds": t1,
                                "iterations": its, "voxel_iters_per_s": its * 16 ** 3 / t1},
            "config2_increment": {"workload": "spheres64 PA66/E-glass, increment 1, Newton-CG", "seconds": t2,
                                  "newton": o2["iterations"], "krylov": o2["krylov"],
                                  "voxel_iters_per_s": pipes2 * 64 ** 3 / t2}}


def batch_bench(nprob=512, steps=5, seed=4, predictor=0):
    """The batched two-scale workload: nprob microproblems of 24^3 / 32^3 / 48^3
    (seeded RSA spheres, own macro histories), all increments, FP32 fields,
    hipGraph chunks, with the uniform or the predictor start. Returns
    Gauss-point updates/s and voxel-iterations/s."""
    import torch

    from paper_2109_14403_amd import hom
    from paper_2109_14403_amd import workloads as W

    wls = [W.batch_problem(i, seed=seed, n_steps=steps) for i in range(nprob)]
    laws = [W.pa66(), W.e_glass()]
    b = hom.Batch([w.phases for w in wls], laws, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP32, tol=1e-6,
                  autotune=1, predictor=predictor)
    nvox = np.array([w.phases.size for w in wls], dtype=np.float64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pipes = np.zeros(nprob)
    failed = 0
    for k in range(steps):
        strains = np.array([w.history[k].strain for w in wls])
        res = b.solve_increment(strains, [w.history[k].theta for w in wls], [w.history[k].grad for w in wls],
                                [w.history[k].dt for w in wls])
        pipes += np.array([r["pipelines"] for r in res])
        failed += sum(1 for r in res if r["status"] != 0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sched = b.schedules()
    b.close()
    sizes = {}
    for w in wls:
        sizes[w.record["n"]] = sizes.get(w.record["n"], 0) + 1
    return {"problems": nprob, "increments": steps, "sizes": {str(k): v for k, v in sorted(sizes.items())},
            "seconds": round(el, 3), "gauss_point_updates_per_s": round(nprob * steps / el, 1),
            "voxel_iters_per_s": round(float((pipes * nvox).sum()) / el, 1), "failed": failed,
            "schedules": sched}


def _hist_args(h, sl=slice(None)):
    steps = h["theta"].shape[1]
    return (h["strain"][sl], h["theta"][sl], np.repeat(h["grad"][sl][:, None], steps, 1),
            np.repeat(h["dt"][sl][:, None], steps, 1))


def surrogate_bench(n_hist=60000, sample=4096, epochs=100, batch=4096, lr=8e-3,
                    runs=((1e-3, 4096), (1e-2, 16384))):
    """Surrogate vs FFT Gauss-point updates/s on the fixed 32^3 microstructure,
    everything inside libhom (hom_surrogate_*): 300k FFT rows (60000
    histories x 5 increments, batched solver, predictor start) train eight
    networks. For each (target, points) in `runs` the threshold is calibrated
    on 6000 fresh histories rolled forward from the networks' own answers so
    that every accepted calibration row meets the target (quantile 1); then fresh
    Gauss points are advanced 5 increments by hom_surrogate_points_step:
    summaries rolled from the surrogate's own answers, rejected points
    answered by the executed FFT fallback (history replay on resident cells).
    The rate is points x increments over the wall time of those calls. The
    first `sample` test points are solved by the FFT solver as the judge; that
    solve also gives the FFT reference rate on the same microstructure."""
    import torch

    from paper_2109_14403_amd import hom
    from paper_2109_14403_amd import workloads as W

    SQ2 = np.sqrt(2.0)
    MW = np.array([1, 1, 1, SQ2, SQ2, SQ2])
    img, _ = W.surrogate_microstructure()
    laws = [W.pa66(), W.e_glass()]
    opts = hom.make_options(precision=hom.FP32, tol=1e-6, predictor=1)
    npts_max = max(p for _, p in runs)
    sur = hom.Surrogate(img, laws, options=opts, n_nets=8, epochs=epochs, batch=batch, lr=lr, target=runs[0][0],
                        quantile=1.0, holdout=0.1, chunk=1024, max_resident=4096)
    hist = W.surrogate_histories(n_hist, seed=10)
    fft, (t_solve, t_setup) = sur.solve_histories(*_hist_args(hist))
    print(f"surrogate: {n_hist * 5} FFT rows in {t_solve:.1f} s (+ {t_setup:.1f} s cell setup)", file=sys.stderr,
          flush=True)
    rep = sur.train(*_hist_args(hist), fft=fft)
    print(f"surrogate: trained {rep}", file=sys.stderr, flush=True)
    # fresh calibration histories (their FFT answers too), the same for every target
    ch = W.surrogate_histories(n_hist // 10, seed=77)
    cfft, _ = sur.solve_histories(*_hist_args(ch))
    th = W.surrogate_histories(npts_max, seed=99)
    truth, (t_ref, _) = sur.solve_histories(*_hist_args(th, slice(0, sample)))
    r_fft = sample * 5 / t_ref
    denom = np.linalg.norm(truth["stress"] * MW, axis=2).max(axis=1)
    # teacher-forced rows of the sample (summaries from the FFT answers), for comparison
    X, _, _ = hom.surrogate_features(*_hist_args(th, slice(0, sample)), truth)
    xd = torch.as_tensor(X, device="cuda")
    out = {
        "fft_gauss_point_updates_per_s": round(r_fft, 1),
        "fft_data_seconds": round(t_solve, 1), "fft_setup_seconds": round(t_setup, 1),
        "train_rows": rep["train_rows"], "fit_seconds": round(rep["fit_seconds"], 1), "epochs": epochs,
        "batch": batch, "networks": 8, "calibration_quantile": 1.0, "holdout_rows": rep["holdout_rows"],
        "median_error_rollout": rep["holdout_median_error"], "median_error_forced": rep["holdout_median_error_forced"],
        "skip_only_median_error": rep["skip_median_error"], "judge_sample_points": sample,
    }
    for target, points in runs:
        cal = sur.calibrate(*_hist_args(ch), cfft, target, 1.0)
        yf, af = sur.infer(xd)
        torch.cuda.synchronize()
        yf, af = yf.cpu().numpy().reshape(sample, 5, 10), af.cpu().numpy().reshape(sample, 5).astype(bool)
        e_forced = np.linalg.norm(yf[:, :, :6] - truth["stress"] * MW, axis=2) / denom[:, None]
        pts = sur.points(points)
        infos, outs, accs = [], [], []
        ok = True
        t0 = time.perf_counter()
        for k in range(5):
            o, acc, info = pts.step(th["strain"][:points, k], th["theta"][:points, k], th["grad"][:points],
                                    th["dt"][:points], check=False)
            print(f"surrogate: target {target:g}, {points} points, step {k}: {info}", file=sys.stderr, flush=True)
            infos.append(info)
            outs.append(o["stress"][:sample].copy())
            accs.append(acc.copy())
            ok = ok and bool((o["status"] == hom.HOM_OK).all())
        t_run = time.perf_counter() - t0
        del pts
        rate = points * 5 / t_run
        acc_all = np.stack(accs, axis=1)
        acc_s = acc_all[:sample]
        e_roll = np.linalg.norm((np.stack(outs, axis=1) - truth["stress"]) * MW, axis=2) / denom[:, None]
        ea, ef = e_roll[acc_s], e_roll[~acc_s]
        out[f"target_{target:g}"] = {
            "threshold": cal["threshold"], "holdout_accepted": round(cal["holdout_accepted"], 4),
            "holdout_accepted_max_error": cal["holdout_accepted_max_error"],
            "points": points, "increments": 5, "seconds": round(t_run, 3),
            "surrogate_gauss_point_updates_per_s": round(rate, 1), "ratio_vs_fft": round(rate / r_fft, 2),
            "accepted_rows": round(float(acc_all.mean()), 4),
            "points_handed_to_fft": int((~acc_all).any(axis=1).sum()),
            "network_ms": round(sum(i["network_ms"] for i in infos), 1),
            "fallback_ms": round(sum(i["fallback_ms"] for i in infos), 1),
            "replayed_increments": int(sum(i["replayed_increments"] for i in infos)),
            "all_status_ok": ok,
            "rolled_accepted_max_error": float(ea.max()) if ea.size else None,
            "rolled_accepted_p99_error": float(np.quantile(ea, 0.99)) if ea.size else None,
            "rolled_accepted_median_error": float(np.median(ea)) if ea.size else None,
            "rolled_accepted_share_within_target": float((ea <= target).mean()) if ea.size else None,
            "fallback_rows_max_error": float(ef.max()) if ef.size else None,
            "forced_accepted": round(float(af.mean()), 4),
            "forced_accepted_max_error": float(e_forced[af].max()) if af.any() else None,
            "forced_median_error": float(np.median(e_forced)),
        }
        print(f"surrogate: {out[f'target_{target:g}']}", file=sys.stderr, flush=True)
    return out


def _counter_rows(folder):
    import csv
    import glob
    rows = []
    for path in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
        with open(path, newline="") as f:
            rows += list(csv.DictReader(f))
    if not rows:
        raise SystemExit(f"no counter_collection.csv under {folder}")
    return rows


def _per_kernel(rows, counter):
    """{kernel name: [values per dispatch]} of one counter (KiB per dispatch)."""
    out = {}
    for r in rows:
        if r["Counter_Name"] == counter:
            out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def pmc_summary(dirs, n, command):
    """Turn rocprofv3 --pmc runs into HBM bytes per launch of each mechanical
    pipeline kernel. dirs = (FETCH_SIZE run, WRITE_SIZE run[, request-size
    run]). Each counter is scaled by what it reads for the 1 GiB calibration
    kernel (torch's elementwise multiply, 1 GiB read + 1 GiB written). The
    optional request-size run (TCC_EA0_RDREQ_32B/_64B/_128B) gives the read
    bytes directly: FETCH_SIZE prices a request as 64 bytes unless the
    TCC_BUBBLE counter flags it as 128 bytes."""
    fetch = _per_kernel(_counter_rows(dirs[0]), "FETCH_SIZE")
    write = _per_kernel(_counter_rows(dirs[1]), "WRITE_SIZE")
    req = None
    if len(dirs) > 2:
        rows = _counter_rows(dirs[2])
        req = {c: _per_kernel(rows, c) for c in ("TCC_EA0_RDREQ_32B", "TCC_EA0_RDREQ_64B", "TCC_EA0_RDREQ_128B")}
    calib_bytes = CALIB_FLOATS * 4

    def calib_name(table):
        cand = [k for k in table if "hom::" not in k and "elementwise" in k.lower()]
        if not cand:
            raise SystemExit("calibration kernel missing: run bench.py with --calib-copy")
        return max(cand, key=lambda k: max(table[k]))

    fscale = calib_bytes / (max(fetch[calib_name(fetch)]) * 1024.0)
    wscale = calib_bytes / (max(write[calib_name(write)]) * 1024.0)

    def req_bytes(name):
        if req is None or name not in req["TCC_EA0_RDREQ_32B"]:
            return None
        return float(32 * np.mean(req["TCC_EA0_RDREQ_32B"][name]) + 64 * np.mean(req["TCC_EA0_RDREQ_64B"][name])
                     + 128 * np.mean(req["TCC_EA0_RDREQ_128B"][name]))

    h = kernel_source_hash()
    lines = [f"# HBM traffic of the pipeline kernels, {n}^3 fibre composite", "",
             f"command: {command}", f"kernel source hash: {h}",
             f"calibration kernel: 1 GiB read + 1 GiB write; FETCH_SIZE scale {fscale:.4f}, "
             f"WRITE_SIZE scale {wscale:.4f}"]
    if req is not None:
        cn = calib_name(req["TCC_EA0_RDREQ_128B"])
        lines.append(f"calibration kernel read bytes by request size: {req_bytes(cn) / calib_bytes:.4f} x 1 GiB")
    lines += ["", "MB per working launch of the mechanical instance (launches that moved at least 5 % of the "
              "kernel's largest launch; a launch of a problem that is not iterating returns at once):", "",
              "| kernel | launches | FETCH raw | WRITE raw | HBM (scaled FETCH + scaled WRITE) | reads by request size |",
              "|---|---|---|---|---|---|"]
    for kind, name in PMC_KINDS.items():
        groups = [k for k in fetch if name in k and "hom::" in k]
        if not groups:
            continue
        # the mechanical instance: the most launches, and the 6-component one
        # where the conduction instance has as many (init, commit)
        main_name = max(groups, key=lambda k: (len(fetch[k]), ", 6>" in k))
        fv = np.asarray(fetch[main_name], dtype=np.float64)
        work = fv >= 0.05 * fv.max() if fv.size else fv > 0

        def avg(table, nm):
            v = np.asarray(table.get(nm, [0.0]), dtype=np.float64)
            return float(np.mean(v[work])) if v.size == work.size else float(np.mean(v))

        f = avg(fetch, main_name) * 1024.0
        w = avg(write, main_name) * 1024.0
        tot = f * fscale + w * wscale
        rb = None
        if req is not None and main_name in req["TCC_EA0_RDREQ_32B"]:
            rb = 32 * avg(req["TCC_EA0_RDREQ_32B"], main_name) + 64 * avg(req["TCC_EA0_RDREQ_64B"], main_name) \
                + 128 * avg(req["TCC_EA0_RDREQ_128B"], main_name)
        rec = {"source_hash": h, "bytes_per_launch": tot, "fetch_bytes_raw": f, "write_bytes_raw": w,
               "fetch_scale": fscale, "write_scale": wscale, "read_bytes_by_request_size": rb,
               "launches": len(fetch[main_name]), "working_launches": int(work.sum()), "kernel": main_name,
               "command": command}
        with open(os.path.join(ROOT, "profiles", f"{kind}_fibres{n}_pmc.json"), "w") as fo:
            json.dump(rec, fo, indent=1)
        rbs = f"{rb / 1e6:.1f}" if rb is not None else "-"
        lines.append(f"| {kind} | {int(work.sum())} of {len(fetch[main_name])} | {f / 1e6:.1f} | {w / 1e6:.1f} | "
                     f"{tot / 1e6:.1f} | {rbs} |")
    with open(os.path.join(ROOT, "profiles", f"pipeline_fibres{n}_hbm_traffic.md"), "w") as fo:
        fo.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def copy_probe(reps=20):
    """Streaming rate of a plain 1 GiB read + 1 GiB write kernel (torch's
    elementwise multiply), GB/s: what a pure streaming kernel reaches here."""
    import torch
    a = torch.ones(CALIB_FLOATS, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 1.0, out=b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.mul(a, 1.0, out=b)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return round(2 * CALIB_FLOATS * 4 / (ms * 1e-3) / 1e9, 1)


def trace_summary(folder, log_path, n, command):
    """rocprofv3 --kernel-trace --stats of a bench run: the stats table, and
    the average duration of the roofline kernel over the launches bench timed
    with events (the last ones of its replayed increments) beside bench's own."""
    import csv
    import glob
    stats = list(csv.DictReader(open(glob.glob(os.path.join(folder, "**", "*kernel_stats.csv"), recursive=True)[0])))
    trace = list(csv.DictReader(open(glob.glob(os.path.join(folder, "**", "*kernel_trace.csv"), recursive=True)[0])))
    with open(log_path) as f:
        d = json.loads([l for l in f if l.startswith("{") and '"metric"' in l][-1])
    roof = d["roofline"]
    kind = roof["kernel"]
    name_part = {"xfwd": "k_xfwd", "xinv": "k_xinv", "zgreen": "k_zgreen", "eval": "k_eval",
                 "yfwd": "k_ypass", "yinv": "k_ypass"}[kind]
    bench_launches = d["kernel_ms"][kind][0]
    rows = [r for r in trace if name_part in r["Kernel_Name"] and "hom::" in r["Kernel_Name"]]
    names = {}
    for r in rows:
        names.setdefault(r["Kernel_Name"], []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    main_name = max(names, key=lambda k: len(names[k]))
    durs = names[main_name]
    if kind in ("yfwd", "yinv"):
        durs = durs[::2] if kind == "yfwd" else durs[1::2]
    tail = durs[-bench_launches:]
    rp_ms = float(np.mean(tail)) / 1e6
    lines = [f"# Kernel trace of the {n}^3 fibre-composite bench", "", f"command: {command}", "",
             f"bench line: value {d['value']:.4g} {d['unit']}, {d['ms_per_step']} ms per increment", "",
             f"roofline kernel `{kind}` ({main_name}):",
             f"- bench (HIP events over its {bench_launches} replayed timed launches): {roof['avg_launch_ms']:.4f} ms",
             f"- rocprofv3 (same {len(tail)} launches): {rp_ms:.4f} ms "
             f"({(rp_ms / roof['avg_launch_ms'] - 1) * 100:+.1f} %)",
             f"- rocprofv3 (all {len(durs)} launches of the run): {float(np.mean(durs)) / 1e6:.4f} ms", "",
             "| kernel | calls | total ms | average us | % |", "|---|---|---|---|---|"]
    for r in stats[:16]:
        lines.append(f"| {r['Name'][:80]} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    # copies inside the timed increments: between the first and the last
    # launch of the roofline kernel, on the queue that runs it
    ev = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"], r["Queue_Id"])
                for r in trace)
    first = next(e for e in ev if e[2] == main_name)
    last = [e for e in ev if e[2] == main_name][-1]
    cps = [e for e in ev if "copyBuffer" in e[2] and first[0] <= e[0] <= last[1]]
    same_q = [e for e in cps if e[3] == first[3]]
    lines += ["", f"`__amd_rocclr_copyBuffer` inside the window of the {len(durs)} `{kind}` launches: "
              f"{len(cps)} copies, {sum(e[1] - e[0] for e in cps) / 1e6:.1f} ms; on the queue of the pipeline "
              f"kernels {len(same_q)} ({sum(e[1] - e[0] for e in same_q) / 1e6:.1f} ms: the per-chunk readback "
              "of the control words). The rest are the checkpoint download before the per-kernel replay "
              "and its restore, outside the timed increments."]
    with open(os.path.join(ROOT, "profiles", f"pipeline_fibres{n}_kernel_trace.md"), "w") as fo:
        fo.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def kernel_table(folder, out_name, title, command, note="", top=20):
    """Top kernels of a rocprofv3 --kernel-trace --stats run as a markdown
    table under profiles/ (calls, total, average and largest launch)."""
    import csv
    import glob
    stats = list(csv.DictReader(open(glob.glob(os.path.join(folder, "**", "*kernel_stats.csv"), recursive=True)[0])))
    homk = [r for r in stats if "hom::" in r["Name"]]
    tot = sum(float(r["TotalDurationNs"]) for r in homk) / 1e6
    lines = [f"# {title}", "", f"command: {command}", ""]
    if note:
        lines += [note, ""]
    lines += [f"hom kernels in total: {tot:.1f} ms ({len(homk)} kernel instances); the {min(top, len(homk))} largest:",
              "", "| kernel | calls | total ms | average us | max us |", "|---|---|---|---|---|"]
    for r in homk[:top]:
        name = r["Name"].replace("void ", "").replace("hom::", "").split("(")[0]
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.1f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} |")
    with open(os.path.join(ROOT, "profiles", out_name), "w") as fo:
        fo.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def network_only(rows=65536, reps=50):
    """Two-network surrogate inference (random weights: the speed does not
    depend on their values) on one 65,536-row batch; prints ms and TFLOP/s."""
    import torch

    from paper_2109_14403_amd import hom
    nets = [hom.MLP(32, 10, seed=s) for s in (0, 1)]
    x = torch.randn(rows, 32, device="cuda")
    for _ in range(5):
        hom.mlp_ensemble_infer(nets, x, 0.0, 1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        hom.mlp_ensemble_infer(nets, x, 0.0, 1.0)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    flops = 2 * rows * 2 * NETWORK_PARAMS_MACS
    print(json.dumps({"rows": rows, "infer_ms": round(ms, 4), "network_tflops": round(flops / (ms * 1e-3) / 1e12, 2)}))


def mfma_summary(folder, command):
    """MFMA busy fraction of the network kernels from one rocprofv3 --pmc run
    with SQ_VALU_MFMA_BUSY_CYCLES (summed over all 1024 SIMDs) and
    GRBM_GUI_ACTIVE (the CSV holds the sum over the 8 XCDs; rocprofv3's own
    MfmaUtil takes the per-XCD value)."""
    rows = _counter_rows(folder)
    busy = _per_kernel(rows, "SQ_VALU_MFMA_BUSY_CYCLES")
    active = _per_kernel(rows, "GRBM_GUI_ACTIVE")
    lines = ["# MFMA utilisation of the surrogate network kernels (65,536-row two-network inference)", "",
             f"command: {command}", "",
             "MfmaUtil = SQ_VALU_MFMA_BUSY_CYCLES / ((GRBM_GUI_ACTIVE / 8 XCDs) x 1024 SIMDs)", "",
             "| kernel | launches | MFMA busy cycles | GUI active cycles per XCD | MfmaUtil % |", "|---|---|---|---|---|"]
    for k in sorted(busy):
        if "mlp" not in k or k not in active:
            continue
        b, a = float(np.mean(busy[k])), float(np.mean(active[k])) / 8
        lines.append(f"| {k[:70]} | {len(busy[k])} | {b:.4g} | {a:.4g} | {b / (a * 1024) * 100:.1f} |")
    with open(os.path.join(ROOT, "profiles", "mlp_infer65536_mfma.md"), "w") as fo:
        fo.write("\n".join(lines) + "\n")
    print("\n".join(lines))


PASS_COUNTERS = ("SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE", "SQ_INSTS_LDS", "SQ_WAIT_INST_LDS",
                 "SQ_ACTIVE_INST_VALU", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "GRBM_GUI_ACTIVE")


def pass_counter_summary(folder, command, out_path=None):
    """LDS and VALU counters of the four FFT pass kernels from one rocprofv3
    --pmc run with PASS_COUNTERS. Derived figures follow rocprofv3's own
    metric definitions, with GRBM_GUI_ACTIVE taken per XCD (the CSV holds the
    sum over the 8 XCDs) and 256 compute units:
    LdsBankConflict = bank-conflict cycles / (LDS active cycles - bank-conflict cycles),
    LdsUtil = LDS active cycles / (GUI active x 256), VALUBusy = VALU active
    cycles / (GUI active x 256), and the share of wave cycles spent waiting to
    issue an LDS instruction."""
    rows = _counter_rows(folder)
    per = {c: _per_kernel(rows, c) for c in PASS_COUNTERS}
    lines = ["# LDS and VALU counters of the FFT pass kernels (256^3 fibre composite, FP32 fields)", "",
             f"command: {command}", "",
             "Per launch, averaged over the run's launches of each kernel. LdsBankConflict = SQ_LDS_BANK_CONFLICT / "
             "(SQ_LDS_IDX_ACTIVE - SQ_LDS_BANK_CONFLICT); LdsUtil = SQ_LDS_IDX_ACTIVE / (GUI x 256 CUs); "
             "VALUBusy = SQ_ACTIVE_INST_VALU / (GUI x 256 CUs); GUI = GRBM_GUI_ACTIVE / 8 XCDs; "
             "LDS wait = SQ_WAIT_INST_LDS / SQ_WAVE_CYCLES.", "",
             "| kernel | launches | LDS instructions | LdsBankConflict | LdsUtil % | VALUBusy % | LDS wait % | "
             "GUI cycles per XCD |", "|---|---|---|---|---|---|---|---|"]
    names = [k for k in per["GRBM_GUI_ACTIVE"]
             if any(p in k for p in ("k_xfwd<float, 6", "k_ypass<float, 6", "k_zgreen<float, 6", "k_xinv<float, 6"))]
    for k in sorted(names):
        if any(k not in per[c] for c in PASS_COUNTERS):
            continue
        m = {c: float(np.mean(per[c][k])) for c in PASS_COUNTERS}
        gui = m["GRBM_GUI_ACTIVE"] / 8
        conf = m["SQ_LDS_BANK_CONFLICT"] / max(m["SQ_LDS_IDX_ACTIVE"] - m["SQ_LDS_BANK_CONFLICT"], 1.0)
        lines.append(f"| {k.split('(')[0].replace('void ', '')} | {len(per['GRBM_GUI_ACTIVE'][k])} | "
                     f"{m['SQ_INSTS_LDS']:.4g} | {conf:.3f} | {100 * m['SQ_LDS_IDX_ACTIVE'] / (gui * 256):.1f} | "
                     f"{100 * m['SQ_ACTIVE_INST_VALU'] / (gui * 256):.1f} | "
                     f"{100 * m['SQ_WAIT_INST_LDS'] / max(m['SQ_WAVE_CYCLES'], 1.0):.1f} | {gui:.4g} |")
    out_path = out_path or os.path.join(ROOT, "profiles", "pipeline_fibres256_lds_valu.md")
    with open(out_path, "w") as fo:
        fo.write("\n".join(lines) + "\n")
    print("\n".join(lines))
    return lines


def dmn_bench(n=128, samples=160, epochs=3000, K=8, points=4096, seed=7):
    """The direct DMN pipeline of Sec. 3 on one fibre microstructure:
    stiffness samples -> effective stiffnesses by the FFT solver (FP32,
    linear elastic, d<sigma>/dE of one increment) -> offline training ->
    online evaluation of many Gauss points with PA66 / E-glass leaves, and the
    DMN's effective stress against the FFT solver on a uniaxial history."""
    import torch
    from paper_2109_14403_amd import hom
    from paper_2109_14403_amd import workloads as W
    rng = np.random.default_rng(seed)
    wl = W.fibre_composite_workload(n, seed=3)          # phase 0 matrix, phase 1 fibres
    w = np.array([1, 1, 1, np.sqrt(2), np.sqrt(2), np.sqrt(2)])

    def te(E, nu):
        return dict(kind="thermoelastic", E=float(E), nu=float(nu), alpha0=0.0, kappa0=1.0, c0=1.0, theta0=293.15)

    def iso(E, nu):
        K, G = E / (3 * (1 - 2 * nu)), E / (2 * (1 + nu))
        P1 = np.zeros((6, 6))
        P1[:3, :3] = 1.0 / 3.0
        return 3 * K * P1 + 2 * G * (np.eye(6) - P1)

    C1, C2, Ce = [], [], []
    t0 = time.perf_counter()
    ctx = hom.Context(wl.phases, [te(1e3, 0.3), te(1e4, 0.3)], scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP32,
                      tol=1e-6)
    for _ in range(samples):      # one context, new law parameters per sample
        E1, nu1 = 10 ** rng.uniform(4.0, 5.2), rng.uniform(0.15, 0.35)      # fibres
        E2, nu2 = 10 ** rng.uniform(1.5, 4.0), rng.uniform(0.30, 0.45)      # matrix
        ctx.set_laws([te(E2, nu2), te(E1, nu1)])
        ctx.solve_increment(np.zeros(6), 293.15, [0, 0, 0], 1.0)
        t = ctx.algorithmic_tangent(what=0)["dsde"]
        C1.append(iso(E1, nu1))
        C2.append(iso(E2, nu2))
        Ce.append(t * w[:, None] / w[None, :])
        if len(Ce) % 40 == 0:
            print(f"dmn samples: {len(Ce)} of {samples}, {time.perf_counter() - t0:.1f} s", file=sys.stderr,
                  flush=True)
    ctx.close()
    fft_s = time.perf_counter() - t0
    C1, C2, Ce = np.array(C1), np.array(C2), np.array(Ce)
    ntr = int(0.9 * samples)
    net = hom.Dmn(K, seed=seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = net.train(C1[:ntr], C2[:ntr], Ce[:ntr], epochs=epochs, batch=32, seed=seed)
    train_s = time.perf_counter() - t0

    def err(a, b):
        return float(np.mean(np.abs(a - b).sum(axis=(1, 2)) / np.abs(b).sum(axis=(1, 2))))

    e_tr = err(net.homogenize(C1[:ntr], C2[:ntr]), Ce[:ntr])
    e_va = err(net.homogenize(C1[ntr:], C2[ntr:]), Ce[ntr:])
    # online: many Gauss points, 5 increments of random proportional loadings
    on = hom.DmnOnline(net, W.e_glass(), W.pa66(), points, tol=1e-8, maxit=30)
    dirs = rng.standard_normal((points, 6))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    steps_t = []
    iters = []
    failed = 0
    for k in range(1, 6):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = on.step(dirs * 0.004 * k, 293.15 + 5 * k, 2.0)
        steps_t.append(time.perf_counter() - t0)
        iters += [r["newton_iters"] for r in out]
        failed += sum(r["status"] != 0 for r in out)
    # the same increments with the predictor start of the jumps
    onp = hom.DmnOnline(net, W.e_glass(), W.pa66(), points, tol=1e-8, maxit=30, predictor=True)
    steps_p, iters_p = [], []
    for k in range(1, 6):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outp = onp.step(dirs * 0.004 * k, 293.15 + 5 * k, 2.0)
        steps_p.append(time.perf_counter() - t0)
        iters_p += [r["newton_iters"] for r in outp]
    onp.close()
    # all four algorithmic tangents at every point: a trial increment (commits nothing)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out4 = on.step(dirs * 0.024, 293.15 + 30, 2.0, what=1, trial=True)
    t_what1 = time.perf_counter() - t0
    failed4 = int((out4["status"] != 0).sum())
    on.close()
    # the DMN against the FFT solver on the first increments of a uniaxial history
    ctx = hom.Context(wl.phases, wl.laws, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP32, tol=1e-6)
    one = hom.DmnOnline(net, W.e_glass(), W.pa66(), 1, tol=1e-8, maxit=30)
    errs = []
    for st in wl.history[:10]:
        f = ctx.solve_increment(st.strain, st.theta, st.grad, st.dt)
        d = one.step(np.asarray(st.strain)[None], st.theta, st.dt)[0]
        errs.append(float(np.abs(d["stress"] - f["stress"]).max() / np.abs(f["stress"]).max()))
    # the effective tangents after the 10th increment: DMN against the FFT solver
    tf = ctx.algorithmic_tangent(what=0)["dsde"]
    tan_err = float(np.abs(d["dsde"] - tf).max() / np.abs(tf).max())
    ctx.close()
    one.close()
    net.close()
    return {"K": K, "grid": n, "samples": samples, "fft_seconds": round(fft_s, 2), "epochs": epochs,
            "train_seconds": round(train_s, 2), "train_loss_first_last": [float(hist[0]), float(hist[-1])],
            "train_mean_error": round(e_tr, 5), "validation_mean_error": round(e_va, 5),
            "online_points": points, "online_ms_per_increment": round(1e3 * float(np.median(steps_t)), 3),
            "online_gauss_point_updates_per_s": round(points / float(np.median(steps_t)), 1),
            "online_newton_mean": round(float(np.mean(iters)), 2), "online_failed": int(failed),
            "online_all_tangents_ms": round(1e3 * t_what1, 3), "online_all_tangents_failed": failed4,
            "online_predictor_ms_per_increment": round(1e3 * float(np.median(steps_p)), 3),
            "online_predictor_newton_mean": round(float(np.mean(iters_p)), 2),
            "vs_fft_tangent_error_increment_10": round(tan_err, 4),
            "vs_fft_stress_error_10_increments": [round(e, 4) for e in errs]}


def predictor_bench(wl, warmup, total, results, disc):
    """The timed increments again with the predictor option (start from the
    last committed strain-fluctuation change): time per increment, iterations,
    and the largest stress difference from the uniform-start run."""
    from paper_2109_14403_amd import hom
    ctx = hom.Context(wl.phases, wl.laws, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP32, tol=1e-6,
                      autotune=1, discretization=disc, predictor=1)
    for st in wl.history[:warmup]:
        ctx.solve_increment(st.strain, st.theta, st.grad, st.dt)
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = [ctx.solve_increment(st.strain, st.theta, st.grad, st.dt) for st in wl.history[warmup:total]]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # d<sigma>/dE after the last timed increment (a first call: uniform starts),
    # then after one more increment (started from the first call's solutions)
    tans = []
    for extra in (False, True):
        if extra:
            st = wl.history[total]
            ctx.solve_increment(st.strain, st.theta, st.grad, st.dt)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        t = ctx.algorithmic_tangent(what=0)
        tans.append((time.perf_counter() - t1, t["krylov_iters"]))
    ctx.close()
    steps = total - warmup
    diff = max(float(np.abs(a["stress"] - b["stress"]).max() / np.abs(b["stress"]).max())
               for a, b in zip(out, results))
    return {"ms_per_step": round(el / steps * 1e3, 2),
            "newton_per_step": sum(r["newton_iters"] for r in out) / steps,
            "krylov_per_step": sum(r["krylov_iters"] for r in out) / steps,
            "max_stress_diff_rel": diff,
            "dsde_ms_first_call": round(tans[0][0] * 1e3, 2), "dsde_krylov_first_call": tans[0][1],
            "dsde_ms_warm": round(tans[1][0] * 1e3, 2), "dsde_krylov_warm": tans[1][1]}


def tangent_bench(ctx, wl, nvox, warmup, total):
    """d<sigma>/dE of the last timed increment: six linearized cell solves
    (hom_algorithmic_tangent, what = 0), timed around the synchronous call."""
    t0 = time.perf_counter()
    t = ctx.algorithmic_tangent(what=0)
    el = time.perf_counter() - t0
    return {"dsde_ms": round(el * 1e3, 2), "dsde_solves": t["solves"], "dsde_krylov": t["krylov_iters"],
            "dsde_pipelines": t["pipelines"], "dsde_voxel_iters_per_s": round(t["pipelines"] * nvox / el, 1),
            "increment": total - 1}


def tangent_full_bench(wl, nvox, warmup):
    """All four tangents on a context set up with the tangent option: the
    first warmup + 1 increments (the last one timed, with the point-partials
    pass before its commit), then seven linearized solves."""
    import torch
    from paper_2109_14403_amd import hom
    ctx = hom.Context(wl.phases, wl.laws, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP32, tol=1e-6,
                      autotune=1, tangent=1)
    for st in wl.history[:warmup]:
        ctx.solve_increment(st.strain, st.theta, st.grad, st.dt)
    st = wl.history[warmup]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = ctx.solve_increment(st.strain, st.theta, st.grad, st.dt)
    inc_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    t = ctx.algorithmic_tangent(what=1)
    el = time.perf_counter() - t0
    ctx.close()
    return {"all_ms": round(el * 1e3, 2), "all_solves": t["solves"], "all_krylov": t["krylov_iters"],
            "all_pipelines": t["pipelines"], "increment_with_partials_ms": round(inc_s * 1e3, 2),
            "increment_with_partials_pipelines": r["pipelines"],
            "dsdt": [round(v, 6) for v in t["dsdt"]], "dDdt": t["dDdt"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-tangent", action="store_true")
    ap.add_argument("--rotated", action="store_true", help="rotated finite-difference discretization")
    ap.add_argument("--no-dmn", action="store_true")
    ap.add_argument("--no-predictor", action="store_true")
    ap.add_argument("--chunk", type=int, default=0, help="solver iterations between host checks (0: library default)")
    ap.add_argument("--calib-copy", action="store_true", help="run a 1 GiB device copy (PMC calibration)")
    ap.add_argument("--pmc-summary", nargs="+", metavar="DIR",
                    help="summarize rocprofv3 --pmc output folders (FETCH_SIZE, WRITE_SIZE[, request sizes]) "
                         "into profiles/ (no GPU needed)")
    ap.add_argument("--mfma-summary", metavar="DIR", help="summarize an MFMA --pmc run into profiles/")
    ap.add_argument("--kernel-table", nargs=3, metavar=("DIR", "OUT", "TITLE"),
                    help="top kernels of a --kernel-trace --stats run as profiles/OUT")
    ap.add_argument("--table-note", default="", help="paragraph under the command line of --kernel-table")
    ap.add_argument("--pass-counter-summary", metavar="DIR",
                    help="summarize a --pmc run with the LDS/VALU counters of the FFT passes into profiles/")
    ap.add_argument("--pmc-command", default="", help="command line recorded in the summary")
    ap.add_argument("--trace-summary", nargs=2, metavar=("TRACE_DIR", "LOG"),
                    help="summarize a rocprofv3 --kernel-trace --stats run of bench.py into profiles/")
    ap.add_argument("--network-only", action="store_true", help="time the surrogate network inference alone")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary, args.n, args.pmc_command)
        return
    if args.trace_summary:
        trace_summary(args.trace_summary[0], args.trace_summary[1], args.n, args.pmc_command)
        return
    if args.kernel_table:
        kernel_table(args.kernel_table[0], args.kernel_table[1], args.kernel_table[2], args.pmc_command,
                     args.table_note)
        return
    if args.mfma_summary:
        mfma_summary(args.mfma_summary, args.pmc_command)
        return
    if args.pass_counter_summary:
        pass_counter_summary(args.pass_counter_summary, args.pmc_command)
        return
    if args.network_only:
        network_only()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_2109_14403_amd import hom
    from paper_2109_14403_amd import workloads as W

    t0 = time.perf_counter()
    wl = W.fibre_composite_workload(args.n, seed=3)
    gen_s = time.perf_counter() - t0
    n = args.n
    hist = wl.history
    total = args.warmup + args.steps
    if total > len(hist):
        raise SystemExit(f"at most {len(hist)} increments")

    if args.calib_copy:
        # a plain streaming kernel of known size (reads 1 GiB, writes 1 GiB)
        a = torch.empty(CALIB_FLOATS, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b

    disc = hom.DISC_ROTATED if args.rotated else hom.DISC_COLLOCATION
    ctx = hom.Context(wl.phases, wl.laws, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP32, tol=1e-6,
                      autotune=1, discretization=disc, chunk=args.chunk)
    print(f"setup done: {n}^3, {wl.record['count']} fibres, fraction {wl.record['fraction']:.4f}, "
          f"{ctx.device_bytes() / 2**30:.1f} GiB on device, generator {gen_s:.1f} s", file=sys.stderr, flush=True)

    for k in range(args.warmup):
        st = hist[k]
        r = ctx.solve_increment(st.strain, st.theta, st.grad, st.dt)
        print(f"warmup inc {k}: newton {r['newton_iters']} krylov {r['krylov_iters']}", file=sys.stderr,
              flush=True)

    # checkpoint, so that the timed increments can be replayed with per-kernel events
    state0 = ctx.get_state(as_array=True) if not args.no_profile else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pipes = 0.0
    tpipes = 0.0
    newton = krylov = 0
    results = []
    for k in range(args.warmup, total):
        st = hist[k]
        r = ctx.solve_increment(st.strain, st.theta, st.grad, st.dt)
        pipes += r["pipelines"]
        tpipes += r["thermal_pipelines"]
        newton += r["newton_iters"]
        krylov += r["krylov_iters"]
        results.append(r)
        print(f"inc {k}: newton {r['newton_iters']} krylov {r['krylov_iters']} stress11 {r['stress'][0]:.4f}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    nvox = float(n) ** 3
    value = pipes * nvox / elapsed

    # per-kernel timing: the timed increments again from the checkpoint, each
    # kernel bracketed by HIP events on the library's stream (launched one by
    # one instead of as graphs; same kernels, same work, same iterations)
    roof = None
    kstats = None
    if not args.no_profile:
        ctx.set_state(state0)
        del state0
        ctx.set_profiling(True)
        n_eval = n_cg = n_first = 0
        for k, r0 in zip(range(args.warmup, total), results):
            st = hist[k]
            pr = ctx.solve_increment(st.strain, st.theta, st.grad, st.dt)
            if (pr["newton_iters"], pr["krylov_iters"]) != (r0["newton_iters"], r0["krylov_iters"]):
                print(f"warning: replay of increment {k} took different iterations", file=sys.stderr)
            n_eval += pr["newton_iters"]
            n_cg += pr["krylov_iters"]
            n_first += max(pr["newton_iters"] - 1, 0)   # every Newton step but the converged one runs CG
        kstats = ctx.kernel_stats()
        ctx.set_profiling(False)
        dom = max((k for k in kstats if kstats[k][0] > 0), key=lambda k: kstats[k][1])
        matrix_fraction = float((wl.phases == 0).mean())
        launches, ms = kstats[dom]
        avg_s = ms / launches / 1e3
        mix = algorithmic_bytes(dom, n, 4, matrix_fraction)
        byt = None
        if mix is not None and launches == n_eval + n_cg:
            byt = (n_eval * mix[0] + n_first * mix[1] + (n_cg - n_first) * mix[2]) / launches
        traffic = traffic_req = None
        pmc_path = os.path.join(ROOT, "profiles", f"{dom}_fibres{n}_pmc.json")
        if os.path.exists(pmc_path):
            pm = json.load(open(pmc_path))
            if pm.get("source_hash") == kernel_source_hash():   # counters of the current kernels only
                traffic = pm.get("bytes_per_launch")
                if pm.get("read_bytes_by_request_size") is not None:
                    traffic_req = pm["read_bytes_by_request_size"] + pm["write_bytes_raw"] * pm["write_scale"]
        if byt is not None:
            ach = byt / avg_s / 1e9
            roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "traffic_request_sized": traffic_req, "kernel": dom,
                    "avg_launch_ms": round(avg_s * 1e3, 4), "algorithmic_bytes": byt}
            # the whole coupled solve: algorithmic bytes of every kernel of the
            # timed increments over their wall time (graph replay, not the
            # per-kernel replay)
            thermal = {k[2:]: kstats[k][0] for k in kstats if k.startswith("t.")}
            sb = solve_bytes(n, 4, matrix_fraction, 79, n_eval, n_cg, n_first, args.steps, thermal)
            tot = sum(sb.values())
            roof["solve_frac"] = round(tot / elapsed / HBM_PEAK_GBS, 4)
            roof["solve_gbs"] = round(tot / elapsed, 1)
            roof["solve_gb_per_step"] = round(tot / args.steps, 2)
            roof["solve_gb_by_kernel"] = {k: round(val / args.steps, 2) for k, val in sb.items()}
            # the same with the HBM bytes the counters measured per launch
            # (profiles/*_pmc.json of the current kernel sources), where every
            # per-voxel kernel of the increment has them; the conduction solve
            # keeps its algorithmic bytes
            cb = counter_solve_bytes(n, n_eval, n_cg, args.steps)
            if cb is not None:
                per_step = (cb + sb["conduction"]) / args.steps
                roof["solve_frac_counters"] = round(per_step * args.steps / elapsed / HBM_PEAK_GBS, 4)
                roof["solve_gb_per_step_counters"] = round(per_step, 2)

    tangent = None
    if not args.no_tangent:
        tangent = tangent_bench(ctx, wl, nvox, args.warmup, total)
        print(f"tangent: {tangent}", file=sys.stderr, flush=True)
    schedules = ctx.schedules()
    ctx.close()
    if tangent is not None:
        tangent.update(tangent_full_bench(wl, nvox, args.warmup))
        print(f"tangent (all four): {tangent}", file=sys.stderr, flush=True)
    pred = None
    if not args.no_predictor:
        pred = predictor_bench(wl, args.warmup, total, results, disc)
        print(f"predictor: {pred}", file=sys.stderr, flush=True)
    copy_gbs = copy_probe()
    batch = None
    if not args.no_batch:
        batch = batch_bench()
        bp = batch_bench(predictor=1)
        batch["predictor"] = {k: bp[k] for k in ("seconds", "gauss_point_updates_per_s", "voxel_iters_per_s",
                                                 "failed")}
        print(f"batch: {batch}", file=sys.stderr, flush=True)
    surr = None
    if not args.no_surrogate:
        surr = surrogate_bench()
        print(f"surrogate: {surr}", file=sys.stderr, flush=True)

    dmn_line = None
    if not args.no_dmn:
        dmn_line = dmn_bench()
        print(f"dmn: {dmn_line}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl.phases, wl.laws)

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "voxel-iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"fibres{n}_pa66_glass", "grid": n, "fibres": wl.record["count"],
                   "fibre_fraction": round(wl.record["fraction"], 4), "scheme": "newton-cg",
                   "fields": "fp32", "reductions": "fp64", "tol": 1e-6,
                   "discretization": "rotated" if args.rotated else "collocation",
                   "increments": f"{args.warmup}..{total - 1} of 50"},
        "thermal_voxel_iters_per_s": round(tpipes * nvox / elapsed, 1),
        "newton_per_step": newton / args.steps, "krylov_per_step": krylov / args.steps,
        "roofline": roof, "copy_probe_gbs": copy_gbs, "cpu_baseline": cpu, "batch": batch, "surrogate": surr,
        "tangent": tangent, "dmn": dmn_line, "predictor": pred, "schedules": schedules,
    }
    if kstats:
        line["kernel_ms"] = {k: [v[0], round(v[1], 3)] for k, v in kstats.items() if v[0]}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
