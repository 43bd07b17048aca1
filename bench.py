#!/usr/bin/env python3
"""Benchmark: enhanced MsRSB set-up + solve on one MI355X.

Workload (default): 3D two-point-flux flow on 128^3 cells with layered,
channelised log-permeability (sigma 2.5, 16 sinusoidal channels, 1000x
contrast), coarse blocks of 8^3 cells (4096 coarse nodes), PCG with l1-Jacobi
x2 pre- and post-smoothing to a true relative residual of 1e-8.

One step = the whole hot path on resident inputs: filter + Jacobi operator,
100 restricted smoothing iterations, R = P^T, A_c = R A P, the exact coarse
inverse, and the preconditioned solve from u = 0.  `value` is the seconds per
step of the FP32-basis form (basis, masked SpGEMM and smoother in FP32;
Krylov, row sums and coarse factorisation in FP64); the all-FP64 form and
the adjoint gradient (96^3 log-normal workload: transposed solve + gradient
kernel) are timed beside it, and the other workloads (2D TPFA, 2D MPFA-O,
3D Q1 elasticity, the 96^3 forward solve, the paper's 2D MPFA-O experiment)
are timed as set-up + solve on the GPU.  Assembly, input generation and
uploads happen before the timed regions.

The `roofline` object covers one PCG iteration of the FP32 form (the bulk of
the step): algorithmic bytes of its kernels in the built data layout (see
pcg_iteration_bytes) over the iteration time measured with HIP events on the
library stream.  `roofline_smoothing` does the same for one restricted
smoothing launch.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
       python bench.py --oracle-times    (oracle on every workload; minutes)
"""
import argparse
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MsRSB setup+solve sec to 1e-8 resid (FP32-basis vs FP64); adjoint grad sec"
KMAX = 100
CHECK_EVERY = 10
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the other workloads")
    ap.add_argument("--forms", default="fp32,fp64",
                    help="forms of the 128^3 step to run (profiling runs take one)")
    ap.add_argument("--dims", type=int, nargs=3, default=None, help="override the grid (debug)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (for scaling HBM counters)")
    ap.add_argument("--oracle-times", action="store_true",
                    help="time the CPU oracle on every workload (median of 3, and 1 thread "
                         "for the small ones) and print one JSON line")
    return ap.parse_args()


# ----------------------------------------------------------------------------
# byte models of the built data layout (per launch / per iteration)
# ----------------------------------------------------------------------------

def smoothing_bytes(n, nnz_p, w):
    """One restricted smoothing launch on a symmetric 7-point stencil: J
    stored factored (s_i = -omega / Dhat_ii and the three upper diagonals of
    Ahat, w bytes each), one byte of slot-map index per stencil entry, P's
    values read once and written once (w bytes per pattern entry).  Neighbour
    rows of P are counted once (their rows are the same array)."""
    return n * (4 * w + 7) + 2 * w * nnz_p


def pcg_iteration_bytes(n, nnz_p, nc):
    """One FP32-form PCG iteration with l1-Jacobi x2 pre and post on a
    symmetric 7-point stencil (A stored as its diagonal and three upper
    diagonals: 16 B per row in FP32, 32 B in FP64), box restriction, grid-
    formed prolongation and the packed symmetric coarse inverse; per kernel,
    each array the kernel touches counted once (bytes per fine row unless
    stated):
      update + two pre-sweeps  x r/w 16, p 8, r 8, q 8, r' w 8, A32 16,
                               dinv 4, z2 w 4                         = 72
      residual t = r - A z2    A32 16, r 8, z2 4, t w 4               = 32
      restriction v_c = R t    R values 4 per entry, t 4
      coarse product           packed lower tiles 8 (T(T+1)/2 64^2), partials
      prolongation z2 += P w_c P values 4 per entry, z2 r/w 8
      post-sweep               A32 16, dinv 4, r 8, z 4, z' w 4       = 36
      post-sweep + dots        A32 16, dinv 4, r 8, z 4, z_old 8, z w 8 = 48
      p = z + beta p, q = A p  A64 32, z 8, p 8, p' w 8, q w 8        = 64
      two finishing reductions partials, 8 B per 256 rows each."""
    nt = (nc + 63) // 64
    ntri = nt * (nt + 1) // 2
    per_row = 72 + 32 + 4 + 8 + 36 + 48 + 64
    coarse = ntri * 64 * 64 * 8 + 2 * ntri * 128 * 8 + 8 * nc
    partials = 3 * 8 * ((n + 255) // 256)
    return n * per_row + 8 * nnz_p + coarse + partials


# ----------------------------------------------------------------------------
# committed profile records
# ----------------------------------------------------------------------------

def _sources_match(rec):
    """True when every 'source_sha256_16.<file>' of a record matches the
    current kernel source."""
    keys = [k for k in rec if k.startswith("source_sha256_16.")]
    if not keys:
        return False
    for k in keys:
        src = os.path.join(ROOT, "paper_1912_06934_amd", "csrc", k.split(".", 1)[1])
        if not os.path.exists(src):
            return False
        if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != rec[k]:
            return False
    return True


def profile_record(name):
    """key = value lines of profiles/<name>.txt, or None."""
    path = os.path.join(ROOT, "profiles", f"{name}.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            rec[k.strip()] = v.strip()
    return rec


def traffic_record(name):
    """Measured HBM bytes (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy)
    from a committed counter summary, if taken on the current kernel
    sources; else None."""
    rec = profile_record(name)
    if not rec or not _sources_match(rec):
        return None
    try:
        return float(rec["bytes_per_unit"])
    except (KeyError, ValueError):
        return None


COPY_BYTES = 1 << 30


def copy_calibration():
    """A plain device-to-device copy of COPY_BYTES, three times: the reference
    against which the FETCH_SIZE / WRITE_SIZE counters are scaled."""
    import torch
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": COPY_BYTES, "copy_bytes_written": COPY_BYTES,
                      "launches": 3}), flush=True)


def system_info():
    cpu = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    rocm = None
    try:
        rocm = open("/opt/rocm/.info/version").read().strip()
    except OSError:
        pass
    info = dict(cpu_model=cpu, host_cores=len(os.sched_getaffinity(0)), rocm=rocm)
    try:
        import torch
        if torch.cuda.is_available():
            prop = torch.cuda.get_device_properties(0)
            info["gpu"] = prop.name or ""
            info["gpu_arch"] = getattr(prop, "gcnArchName", "")
            info["gpu_cus"] = prop.multi_processor_count
            info["gpu_mem_gib"] = round(prop.total_memory / 2**30, 1)
            info["torch_hip"] = torch.version.hip
    except Exception:  # pragma: no cover
        pass
    if "Instinct" not in info.get("gpu", ""):
        # the marketing name from the runtime's agent list when torch's is
        # missing or generic
        try:
            out = subprocess.run(["/opt/rocm/bin/rocminfo"], capture_output=True, text=True,
                                 timeout=30).stdout
            names = [l.split(":", 1)[1].strip() for l in out.splitlines()
                     if l.strip().startswith("Marketing Name")]
            gpus = [x for x in names if "Instinct" in x or "MI" in x]
            if gpus:
                info["gpu"] = gpus[0]
        except (OSError, subprocess.SubprocessError):
            pass
    return info


# ----------------------------------------------------------------------------
# GPU runs
# ----------------------------------------------------------------------------

def _median(x):
    return float(np.median(np.asarray(x, dtype=np.float64)))


def run_extra(dev, steps):
    """Set-up + solve of the other workloads on the GPU (median over steps;
    inputs resident, assembled once)."""
    import torch
    import synth
    from paper_1912_06934_amd import Msrsb
    out = {}
    for name in ("c1", "c2", "c3", "c5", "e2"):
        cfg = synth.make_config(name)
        sup = cfg["supports"]
        s = Msrsb(device=0, stream=torch.cuda.current_stream(dev).cuda_stream)
        if cfg["kind"] == "tpfa":
            logk = torch.from_numpy(cfg["logk"]).to(dev)
            f = torch.empty_like(logk)
            s.assemble_tpfa(cfg["dims"], cfg["h"], logk, cfg["bc"], f)
        else:
            rp, ci, a = cfg["matrix"]
            s.set_matrix(rp, ci, a, cfg.get("block_size", 1))
            f = torch.from_numpy(np.ascontiguousarray(cfg["rhs"])).to(dev)
        s.set_coarse(sup["nc"], sup["part"], sup["prp"], sup["pci"], sup["interior"])
        fp32 = name == "c5"          # the differentiation form's FP32 basis
        kw = dict(krylov=cfg["krylov"], pre=cfg["pre"], post=cfg["post"],
                  ordering=cfg["ordering"], rtol=1e-8, max_iter=5000)
        if cfg["krylov"] == "gmres":
            kw["restart"] = cfg["restart"]
        times, iters, res = [], [], []
        for rep in range(1 + steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.setup_basis(max_iter=KMAX, check_every=CHECK_EVERY, fp32_basis=fp32)
            s.build_coarse()
            u = torch.zeros_like(f)
            info = s.solve(f, u, **kw)
            torch.cuda.synchronize()
            if rep:
                times.append(time.perf_counter() - t0)
                iters.append(info["iters"])
                res.append(info["true_rel_res"])
        tm = s.timings()
        out[name] = dict(sec=round(_median(times), 6), n=int(f.numel()), nc=int(sup["nc"]),
                         krylov=cfg["krylov"], iters=int(iters[-1]),
                         true_rel_res=float(max(res)),
                         phases_ms={k: round(v, 3) for k, v in tm.items() if v})
        log(f"{name}: {out[name]['sec'] * 1e3:.2f} ms set-up + solve, {iters[-1]} "
            f"{cfg['krylov']} iterations, res {max(res):.2e}")
        s.close()
    return out


def oracle_times():
    """The CPU oracle on every workload: set-up + solve to 1e-8 with the
    workload's recipe, median of 3 on all host threads, and one run on a
    single thread for the small workloads (c1, c2, e2) and c5."""
    import oracle
    import synth
    info = system_info()
    nthreads = info["host_cores"]

    def run(name):
        cfg = synth.make_config(name)
        sup = cfg["supports"]
        if cfg["kind"] == "tpfa":
            rp, ci, a, f = oracle.tpfa(cfg["dims"], cfg["h"], cfg["logk"], cfg["bc"])
        else:
            rp, ci, a = cfg["matrix"]
            f = cfg["rhs"]
        kw = dict(krylov=cfg["krylov"], pre=cfg["pre"], post=cfg["post"],
                  ordering=cfg["ordering"], rtol=1e-8, maxit=5000)
        if cfg["krylov"] == "gmres":
            kw["restart"] = cfg["restart"]
        t0 = time.perf_counter()
        m = oracle.Msrsb(rp, ci, a, cfg.get("block_size", 1))
        m.set_coarse(sup["nc"], sup["part"], sup["prp"], sup["pci"], sup["interior"])
        m.setup_basis(kmax=KMAX, nit=CHECK_EVERY)
        m.build_coarse()
        r = m.solve(f, **kw)
        return time.perf_counter() - t0, r["iters"]

    out = dict(system=info, threads=nthreads, workloads={})
    for name in ("c1", "c2", "e2", "c3", "c4", "c5"):
        ts, its = [], None
        for _ in range(3):
            dt, its = run(name)
            ts.append(dt)
        rec = dict(median_s=round(_median(ts), 3), runs_s=[round(t, 3) for t in ts], iters=its)
        log(f"oracle {name}: {rec}")
        out["workloads"][name] = rec
    # single-thread runs in child processes (OMP_NUM_THREADS is read at start-up)
    for name in ("c1", "c2", "e2", "c5"):
        env = dict(os.environ, OMP_NUM_THREADS="1")
        code = ("import sys, json; sys.path.insert(0, %r); import bench; "
                "print(json.dumps(bench._oracle_one(%r)))" % (ROOT, name))
        res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                             text=True, check=True)
        rec = json.loads(res.stdout.strip().splitlines()[-1])
        out["workloads"][name]["one_thread_s"] = rec["sec"]
        log(f"oracle {name} on one thread: {rec['sec']:.3f} s")
    print(json.dumps(out), flush=True)


def _oracle_one(name):
    import oracle
    import synth
    cfg = synth.make_config(name)
    sup = cfg["supports"]
    if cfg["kind"] == "tpfa":
        rp, ci, a, f = oracle.tpfa(cfg["dims"], cfg["h"], cfg["logk"], cfg["bc"])
    else:
        rp, ci, a = cfg["matrix"]
        f = cfg["rhs"]
    kw = dict(krylov=cfg["krylov"], pre=cfg["pre"], post=cfg["post"], ordering=cfg["ordering"],
              rtol=1e-8, maxit=5000)
    if cfg["krylov"] == "gmres":
        kw["restart"] = cfg["restart"]
    t0 = time.perf_counter()
    m = oracle.Msrsb(rp, ci, a, cfg.get("block_size", 1))
    m.set_coarse(sup["nc"], sup["part"], sup["prp"], sup["pci"], sup["interior"])
    m.setup_basis(kmax=KMAX, nit=CHECK_EVERY)
    m.build_coarse()
    r = m.solve(f, **kw)
    return dict(sec=round(time.perf_counter() - t0, 3), iters=r["iters"],
                threads=oracle.threads())


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.oracle_times:
        oracle_times()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "decomposition is a design note, not a built path.", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    from paper_1912_06934_amd import Msrsb

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)

    # ---------------- inputs (untimed) ----------------
    t0 = time.time()
    cfg = synth.make_config("c4", dims=args.dims)
    dims, h, bc = cfg["dims"], cfg["h"], cfg["bc"]
    n = int(np.prod(dims))
    sup = cfg["supports"]
    logk = torch.from_numpy(cfg["logk"]).to(dev)
    rhs = torch.empty_like(logk)
    log(f"inputs {dims} n={n} nc={sup['nc']} nnz_P={sup['prp'][-1]} ({time.time() - t0:.1f}s)")

    s = Msrsb(device=0, stream=stream.cuda_stream)
    s.assemble_tpfa(dims, h, logk, bc, rhs)
    s.set_coarse(sup["nc"], sup["part"], sup["prp"], sup["pci"], sup["interior"])
    nnz_a = int(s.get_matrix()[0][-1])
    nnz_p = int(sup["prp"][-1])
    nc = int(sup["nc"])
    solve_kw = dict(krylov="pcg", rtol=1e-8, max_iter=2000, pre=(2, 2), post=(2, 2))

    def step(fp32):
        b = s.setup_basis(max_iter=KMAX, check_every=CHECK_EVERY, fp32_basis=fp32)
        s.build_coarse()
        u = torch.zeros_like(rhs)
        info = s.solve(rhs, u, fp32_smoother=fp32, **solve_kw)
        return b, info

    results = {}
    forms = [f for f in ("fp32", "fp64") if f in args.forms.split(",")]
    for form, fp32 in [(f, f == "fp32") for f in forms]:
        for _ in range(args.warmup):
            step(fp32)
        torch.cuda.synchronize()
        smooth_ms, solve_ms, iters, res = [], [], [], []
        t_start = time.perf_counter()
        for _ in range(args.steps):
            b, info = step(fp32)
            tm = s.timings()
            smooth_ms.append(tm["smooth"])
            solve_ms.append(tm["solve"])
            iters.append(info["iters"])
            res.append(info["true_rel_res"])
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t_start) / args.steps
        tm = s.timings()
        results[form] = dict(sec=wall, smooth_ms=float(np.mean(smooth_ms)),
                             solve_ms=float(np.mean(solve_ms)), iters=iters,
                             true_rel_res=max(res), phases=tm)
        log(f"{form}: {wall * 1e3:.2f} ms/step, PCG iters {iters}, res {max(res):.2e}, "
            f"phases(ms) {{{', '.join(f'{k}: {v:.2f}' for k, v in tm.items() if v)}}}")

    # ---------------- adjoint gradient (96^3 workload) ----------------
    adjoint = None
    if not args.no_adjoint:
        from paper_1912_06934_amd import MsrsbTPFASolve, TPFAProblem
        c5 = synth.make_config("c5")
        s5 = c5["supports"]
        prob = TPFAProblem(dims=c5["dims"], h=c5["h"], bc=tuple(c5["bc"]),
                           coarse=dict(nc=s5["nc"], part=s5["part"], prp=s5["prp"],
                                       pci=s5["pci"], interior=s5["interior"]),
                           rtol=1e-8, fp32_basis=True)
        lk = torch.from_numpy(c5["logk"]).to(dev).requires_grad_(True)
        ob = torch.as_tensor(c5["obs"], device=dev)
        dd = torch.as_tensor(c5["data"], device=dev)
        times = []
        for rep in range(args.warmup + args.steps):
            lk.grad = None
            p = MsrsbTPFASolve.apply(lk, prob)
            J = ((p[ob] - dd) ** 2).sum()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            J.backward()
            torch.cuda.synchronize()
            if rep >= args.warmup:
                times.append(time.perf_counter() - t1)
        tm = prob.solver.timings()
        adjoint = dict(sec=float(np.median(times)), solve_t_ms=tm["solve_t"], grad_ms=tm["grad"],
                       iters=prob.last_backward["solve"]["iters"])
        log(f"adjoint: {adjoint}")

    # ---------------- the other workloads ----------------
    extra = None if args.no_extra else run_extra(dev, max(1, min(args.steps, 3)))

    if "fp32" not in results or "fp64" not in results:
        log("profiling run: one form only, no JSON line")
        return

    # ---------------- rooflines ----------------
    fp32 = results["fp32"]
    it32 = fp32["iters"][-1]
    iter_s = fp32["solve_ms"] / 1e3 / it32
    pcg_bytes = pcg_iteration_bytes(n, nnz_p, nc)
    achieved = pcg_bytes / iter_s / 1e9
    roofline = dict(kernel="one PCG iteration, FP32 form: k_pcg_update_sweep2, k_dia_residual, "
                           "k_restrict_box, k_symv_tiles, k_symv_final, k_prolong_axes, "
                           "k_dia_sweep, k_dia_sweep_dots, k_fin_beta, k_pcg_p_spmv_dia, "
                           "k_fin_alpha",
                    bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=traffic_record("pcg_iteration_f32_c4_traffic"),
                    algorithmic_bytes_per_unit=int(pcg_bytes), unit_of_work="PCG iteration",
                    avg_us_per_unit=round(iter_s * 1e6, 2),
                    timing="solve phase (HIP events on the library stream) / iterations")
    sm_s = fp32["smooth_ms"] / KMAX / 1e3
    sm_bytes = smoothing_bytes(n, nnz_p, 4)
    sm_ach = sm_bytes / sm_s / 1e9
    roofline_smoothing = dict(
        kernel="k_smooth_map<float, unsigned char, 8, 7, true, true> (restricted smoothing, "
               "FP32, P split in halves)",
        bound="hbm", achieved=round(sm_ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
        frac=round(sm_ach / HBM_PEAK_GBS, 4), traffic=traffic_record("k_smooth_f32_c4_traffic"),
        algorithmic_bytes_per_unit=int(sm_bytes), unit_of_work="smoothing launch",
        avg_us_per_unit=round(sm_s * 1e6, 2),
        timing="smoothing phase (HIP events) / 100 launches (includes the 10 e_it checks)")

    # ---------------- CPU oracle baseline ----------------
    cpu = None
    if not args.no_cpu:
        import oracle
        rp, ci, a, f = oracle.tpfa(dims, h, cfg["logk"], bc)
        dts = []
        for _ in range(3):
            m = oracle.Msrsb(rp, ci, a)
            m.set_coarse(sup["nc"], sup["part"], sup["prp"], sup["pci"], sup["interior"])
            t1 = time.perf_counter()
            m.setup_basis(kmax=KMAX, nit=CHECK_EVERY)
            m.build_coarse()
            r = m.solve(f, rtol=1e-8, pre=(2, 2), post=(2, 2), maxit=2000)
            dts.append(time.perf_counter() - t1)
        cpu = dict(value=round(_median(dts), 3), unit="s", cores=oracle.threads(), kind="oracle",
                   sample="the full FP64 workload, median of 3 runs: filter, 100 smoothing "
                          "iterations, R A P, dense LU, PCG to 1e-8 "
                          f"({r['iters']} iterations)",
                   runs_s=[round(t, 3) for t in dts])
        log(f"cpu oracle: {cpu}")
    orc_rec = profile_record("oracle_times")
    orc_summary = None
    if orc_rec and "summary" in orc_rec:
        try:
            orc_summary = json.loads(orc_rec["summary"])
        except ValueError:
            orc_summary = None

    fp64 = results["fp64"]
    line = {
        "metric": METRIC, "value": round(fp32["sec"], 5), "unit": "s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(fp32["sec"] * 1e3, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 basis+smoother / f64 krylov+coarse", "data": "synthetic",
        "config": {"workload": f"3D TPFA {'x'.join(map(str, dims))} channelised log-k, "
                               f"8^3 coarse blocks ({nc} coarse), 100 smoothing its, "
                               "PCG + l1-Jacobi x2 pre/post to 1e-8",
                   "n": n, "nnz_A": nnz_a, "nnz_P": nnz_p, "nc": nc},
        "fp64_value": round(fp64["sec"], 5),
        "fp32_pcg_iters": fp32["iters"][-1], "fp64_pcg_iters": fp64["iters"][-1],
        "true_rel_res": max(fp32["true_rel_res"], fp64["true_rel_res"]),
        "phases_ms_fp32": {k: round(v, 3) for k, v in fp32["phases"].items() if v},
        "phases_ms_fp64": {k: round(v, 3) for k, v in fp64["phases"].items() if v},
        "adjoint_grad_s": None if adjoint is None else round(adjoint["sec"], 5),
        "adjoint": adjoint,
        "other_workloads": extra,
        "roofline": roofline,
        "roofline_smoothing": roofline_smoothing,
        "cpu_baseline": cpu,
        "oracle_times": orc_summary,
        "system": system_info(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
