"""Benchmark of the SEM Poisson/Helmholtz hot path on one MI355X.

Step = one application of the assembled operator, sem_ax then sem_gs
(w = QQ^T A_L u), on the 16x16x16 deformed hex box at N=7 (2,097,152 local /
1,442,897 unique points), FP64, all six geometric factors, seeded
uniform[-1,1] input resident in HBM.  value = unique DOFs per second.

Also reported on the same JSON line:
  roofline      the dominant kernel (the FP64 element operator) timed with HIP
                events on the stream it runs on, algorithmic bytes / time
                against the 8 TB/s HBM peak; HBM traffic from the rocprofv3
                counter summary in profiles/ when it matches this kernel source
  cpu_baseline  the CPU oracle (oracle/), timed on this host's cores on a
                bounded sample of the same workload
  ax_three_fields  sem_ax_multi on three fields of the same mesh (the
                geometric factors read once for all three)
  projection    a sequence of slowly varying loads solved from zero and with
                initial guesses projected onto earlier solutions
  pcg           time to a true relative residual of 1e-8 on the 32^3 deformed
                Helmholtz box (h1=1, h2=10, N=7, 3 Gaussian right-hand sides):
                FCG with the FP32 p-multigrid (7->3->1) against FP64 Jacobi-PCG,
                each right-hand side solved on its own and the three in lockstep;
                beside it the element operator alone on that mesh (one field,
                and three through sem_ax_multi), beyond the Infinity Cache
  advection     the dealiased advection operator (Gauss rule exact for degree
                3N) on the 32^3 deformed box, three fields per call, against the
                HBM and FP64 peaks
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

METRIC = "GDOF/s per Ax (N=7 FP64) + PCG time-to-1e-8, mixed-prec vs FP64, %HBM peak"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6  # MI355X dense FP64 (vector and matrix)
AX_BYTES_PER_POINT = 64  # u 8 + six G 48 + w 8 (FP64 Poisson)
AX3_BYTES_PER_POINT = 96  # three fields: 3 x (u 8 + w 8) + six G 48 read once
AX32_BYTES_PER_POINT = 32  # FP32 Poisson: u 4 + six G 24 + w 4
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "ax_fp64_box16_n7_traffic.txt")
AX_SOURCE = os.path.join(ROOT, "paper_2104_05829_amd", "csrc", "ax_impl.h")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def ax_source_sha():
    with open(AX_SOURCE, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the FP64 element operator from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    if not os.path.exists(PROFILE_TRAFFIC):
        return None
    kv = {}
    for line in open(PROFILE_TRAFFIC):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != ax_source_sha():
        return None
    try:
        return float(kv["hbm_bytes_per_launch_scaled"])
    except (KeyError, ValueError):
        return None


_ORACLE_TIMING_DIR = None


def oracle_timing_lib():
    """The oracle's all-core timing build (OpenMP over elements, -O3
    -march=native), compiled on this host into a temporary directory."""
    global _ORACLE_TIMING_DIR
    import tempfile
    import oracle
    if _ORACLE_TIMING_DIR is None:
        _ORACLE_TIMING_DIR = tempfile.mkdtemp(prefix="oracle_omp_")
    return oracle.timing_lib(_ORACLE_TIMING_DIR)


class OracleResidual:
    """True relative residuals ||R (b - QQ^T A_L x)||_W / ||R b||_W of GPU
    solutions, recomputed by the CPU oracle in FP64 from the mesh alone
    (its own GLL nodes, geometric factors, element operator and QQ^T; the
    element loops of the geometry and the operator on all cores through the
    timing build, which computes bit-identical elements)."""

    def __init__(self, mesh, N=7):
        import oracle
        self.oracle = oracle
        self.N = N
        xi, rho = oracle.gll(N)
        self.D = oracle.dhat(N, xi)
        self.lib = oracle_timing_lib()
        self.G, self.B, _ = oracle.geometry(N, mesh.x, mesh.y, mesh.z, self.D, rho, _lib=self.lib)
        self.gid = mesh.gid.reshape(-1)
        mask = 1.0 - mesh.dirichlet.reshape(-1).astype(np.float64)
        self.W = mask / oracle.multiplicity(self.gid)
        self.mask = mask

    def rel(self, x, b, h1, h2):
        o = self.oracle
        Ax = o.qqt(self.gid, o.ax(self.N, self.D, self.G, x, h1=h1, h2=h2, B=self.B, _lib=self.lib))
        r = self.mask * (b - Ax)
        bm = self.mask * b
        return float(np.sqrt(np.sum(self.W * r * r) / np.sum(self.W * bm * bm)))


def bench_operator(args, torch, sem_mod, inputs):
    N = 7
    mesh = sem_mod.box_mesh(16, 16, 16, N, deform="cyclic", amp=0.05, bc="neumann")
    s = sem_mod.Sem(mesh)
    inf = s.info()
    nL, nU = inf["n_local"], inf["n_unique"]
    u = torch.tensor(inputs.uniform_lvector(nL, 2), device="cuda")
    w = torch.empty_like(u)
    for _ in range(args.warmup):
        s.ax(u, w)
        s.gs(w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s.ax(u, w)
        s.gs(w)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    # dominant kernel alone, HIP events on the stream it is launched on
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        s.ax(u, w)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_ax = ev0.elapsed_time(ev1) / args.steps
    ev0.record(stream)
    for _ in range(args.steps):
        s.gs(w)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_gs = ev0.elapsed_time(ev1) / args.steps
    # three fields through one batched operator call (G read once per element)
    U3 = torch.stack([u, torch.flip(u, (0,)), 0.5 * u])
    W3 = torch.empty_like(U3)
    for _ in range(3):
        s.ax_multi(U3, W3)
    ev0.record(stream)
    for _ in range(args.steps):
        s.ax_multi(U3, W3)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_ax3 = ev0.elapsed_time(ev1) / args.steps
    # per-step HIP-event times (median and mean), separately from the timed loop above
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    for a, b_ in evs:
        a.record(stream)
        s.ax(u, w)
        s.gs(w)
        b_.record(stream)
    torch.cuda.synchronize()
    per_step = sorted(a.elapsed_time(b_) for a, b_ in evs)
    s.free()
    # the FP32 form of the same step (the smoother's precision): level 0 of a
    # p-MG handle, sem_ax_level + sem_gs_level in FP32
    s32 = sem_mod.Sem(mesh, levels=(7, 3, 1))
    u32 = u.float()
    w32 = torch.empty_like(u32)
    for _ in range(args.warmup):
        s32.ax_level(0, u32, w32)
        s32.gs_level(0, w32)
    ev0.record(stream)
    for _ in range(args.steps):
        s32.ax_level(0, u32, w32)
        s32.gs_level(0, w32)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_step32 = ev0.elapsed_time(ev1) / args.steps
    ev0.record(stream)
    for _ in range(args.steps):
        s32.ax_level(0, u32, w32)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_ax32 = ev0.elapsed_time(ev1) / args.steps
    s32.free()
    del u32, w32
    # a plain device copy of 1 GiB (torch), the measured stream reference
    x = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(2):
        y.copy_(x)
    ev0.record(stream)
    for _ in range(10):
        y.copy_(x)
    ev1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * x.numel() * 8 / (ev0.elapsed_time(ev1) / 10 * 1e-3) / 1e9
    del x, y
    return dict(mesh=mesh, nL=nL, nU=nU, ms_step=ms_step, ms_ax=ms_ax, ms_gs=ms_gs, ms_ax3=ms_ax3,
                n_shared=inf["n_shared_copies"], n_seg=inf["n_segments"],
                ms_step_median=per_step[len(per_step) // 2], ms_step_mean=sum(per_step) / len(per_step),
                ms_step32=ms_step32, ms_ax32=ms_ax32, copy_gbs=copy_gbs)


def bench_pcg(args, torch, sem_mod, inputs):
    """32^3 deformed box, N=7, h1=1, h2=10, homogeneous Dirichlet; 3 RHS
    f ~ N(0,1) per node (seeds 30, 31, 32), b = QQ^T(B f) assembled on the GPU
    with the library's own mass matrix."""
    N = 7
    ne = args.pcg_elems
    mesh = sem_mod.box_mesh(ne, ne, ne, N, deform="cyclic", amp=0.05, bc="dirichlet")
    t0 = time.perf_counter()
    s = sem_mod.Sem(mesh, levels=(7, 3, 1))
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    _, B = s.geometry()
    W, _ = s.weights()
    pres = ("pmg", "jacobi") if args.pcg_precond == "both" else (args.pcg_precond,)
    res = {pre: [] for pre in pres}
    first_call = {}
    for seed in (30, 31, 32)[: args.pcg_rhs]:
        f = torch.tensor(inputs.gaussian_per_node(mesh.gid, seed), device="cuda")
        b = s.gs(B * f) * (W > 0)
        for pre in pres:
            # first call builds the preconditioner (cached afterwards)
            if not res[pre]:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s.solve(b, tol=1e-8, h1=1.0, h2=10.0, precond=pre, maxit=20000)
                torch.cuda.synchronize()
                first_call[pre] = time.perf_counter() - t0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, st, rc = s.solve(b, tol=1e-8, h1=1.0, h2=10.0, precond=pre, maxit=20000,
                                coarse_tol=args.coarse_tol, coarse_maxit=args.coarse_maxit)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            res[pre].append(dict(seed=seed, ms=dt * 1e3, iters=st["iters"],
                                 true_rel_res=st["true_rel_res"], rc=rc,
                                 coarse_iters=st["coarse_iters"], x=x))
    # the same right-hand sides solved together, in lockstep (one batched
    # operator / gather-scatter per iteration for all unconverged systems)
    lock = {}
    if args.pcg_rhs > 1:
        Bt = torch.stack([s.gs(B * torch.tensor(inputs.gaussian_per_node(mesh.gid, seed), device="cuda"))
                          * (W > 0) for seed in (30, 31, 32)[: args.pcg_rhs]])
        for pre in pres:
            # untimed first lockstep call: grows the solver workspace to the batch
            s.solve_multi(Bt, tol=1e-8, h1=1.0, h2=10.0, precond=pre, maxit=20000,
                          coarse_tol=args.coarse_tol, coarse_maxit=args.coarse_maxit)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            X, sts, rc = s.solve_multi(Bt, tol=1e-8, h1=1.0, h2=10.0, precond=pre, maxit=20000,
                                       coarse_tol=args.coarse_tol, coarse_maxit=args.coarse_maxit)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            dif = [float(torch.sqrt(torch.sum(W * (X[q] - r["x"]) ** 2) / torch.sum(W * r["x"] ** 2)))
                   for q, r in enumerate(res[pre])]
            lock[pre] = {"ms_total": round(dt * 1e3, 3), "iters": [st["iters"] for st in sts],
                         "true_rel_res": [float(f"{st['true_rel_res']:.3e}") for st in sts],
                         "status": rc, "rel_diff_vs_independent": [float(f"{d:.3e}") for d in dif]}
            if pre == "pmg":
                lock[pre]["coarse_iters"] = [st["coarse_iters"] for st in sts]
            del X
    # Schwarz smoothers (CHEBY-ASM / CHEBY-RAS), the three right-hand sides in lockstep
    schw = {}
    schw_x = {}  # solutions of the one-by-one Schwarz solves, for the oracle's residuals
    if "pmg" in pres and not args.no_schwarz:
        Bt = torch.stack([s.gs(B * torch.tensor(inputs.gaussian_per_node(mesh.gid, seed), device="cuda"))
                          * (W > 0) for seed in (30, 31, 32)[: args.pcg_rhs]])
        for smo in ("asm", "ras"):
            kw = dict(tol=1e-8, h1=1.0, h2=10.0, precond="pmg", smoother=smo, cheb_lo=0.25,
                      coarse_tol=args.coarse_tol, coarse_maxit=args.coarse_maxit)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.solve_multi(Bt, **kw)  # builds the smoother (host FDM setup) and its lambda_max
            torch.cuda.synchronize()
            t_setup = time.perf_counter() - t0
            t0 = time.perf_counter()
            X, sts, rc = s.solve_multi(Bt, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            schw[smo] = {"ms_total": round(dt * 1e3, 3), "iters": [st["iters"] for st in sts],
                         "true_rel_res": [float(f"{st['true_rel_res']:.3e}") for st in sts],
                         "status": rc, "first_call_s": round(t_setup, 3)}
            del X
            # the same right-hand sides solved one by one (as the CHEBY-JAC
            # p-MG record "pmg" solves them)
            single = []
            for q in range(Bt.shape[0]):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                xq, st, rcq = s.solve(Bt[q], **kw)
                torch.cuda.synchronize()
                single.append(((time.perf_counter() - t0) * 1e3, st["iters"], st["true_rel_res"], rcq))
                if not args.no_cpu:
                    schw_x.setdefault(smo, []).append((xq.cpu().numpy(), Bt[q].cpu().numpy()))
                del xq
            schw[smo + "_single"] = {"ms_per_rhs": [round(t[0], 3) for t in single],
                                     "iters": [t[1] for t in single],
                                     "true_rel_res": [float(f"{t[2]:.3e}") for t in single],
                                     "status": [t[3] for t in single]}
        # one level-0 ASM application (FDM solves, extension combine, QQ^T,
        # weight) on one FP32 field, HIP events; the oracle's Schwarz operator
        # on the 5x5x5 block at the mesh corner, one thread, scaled per element
        r32 = Bt[0].float()
        z32 = s.smoother_apply(0, r32, smoother="asm", h1=1.0, h2=10.0)
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(10):
            s.smoother_apply(0, r32, z32, smoother="asm", h1=1.0, h2=10.0)
        e1.record(stream)
        torch.cuda.synchronize()
        schw["apply"] = {"call": "sem_smoother_apply level 0 (N=7), ASM, one FP32 field",
                         "ms": round(e0.elapsed_time(e1) / 10, 4)}
        if not args.no_cpu:
            from threadpoolctl import threadpool_limits
            from oracle import asm as oasm, solvers as osol
            nqq = N + 1
            idx = np.array([ex + ne * (ey + ne * ez) for ez in range(5) for ey in range(5) for ex in range(5)])
            sub = inputs.BoxMesh(N=N, shape=(5, 5, 5), x=mesh.x[idx], y=mesh.y[idx], z=mesh.z[idx],
                                 gid=mesh.gid[idx], dirichlet=mesh.dirichlet[idx])
            with threadpool_limits(limits=1):
                lv = osol.Level(N, sub.x, sub.y, sub.z, sub.gid, sub.dirichlet, 1.0, 10.0)
                O = oasm.Schwarz(lv, sub.shape, sub.x, sub.y, sub.z, sub.dirichlet, "asm")
                rs = r32.cpu().numpy().reshape(-1, nqq ** 3)[idx].reshape(-1).astype(np.float64)
                t0 = time.perf_counter()
                O.apply(rs)
                dt = time.perf_counter() - t0
            schw["apply"]["cpu_oracle"] = {"kind": "oracle", "cores": 1,
                                           "sample": "the 5x5x5 corner block (125 elements), numpy one thread, "
                                                     "scaled per element",
                                           "ms_scaled": round(dt * 1e3 * mesh.E / 125, 1)}
    # phase breakdown of one more solve of the first right-hand side with the
    # library's event timers (not part of the timed solves above)
    phases = {}
    b0 = s.gs(B * torch.tensor(inputs.gaussian_per_node(mesh.gid, 30), device="cuda")) * (W > 0)
    for pre in pres:
        _, st, _ = s.solve(b0, tol=1e-8, h1=1.0, h2=10.0, precond=pre, maxit=20000, timers=1,
                           coarse_tol=args.coarse_tol, coarse_maxit=args.coarse_maxit)
        phases[pre] = {k: round(st[k], 3) for k in ("ms_ax", "ms_gs", "ms_vec", "ms_prec", "ms_coarse")}
        phases[pre]["ms_solve"] = round(st["ms_solve"], 3)
    # the element operator alone on this mesh (out of the 256 MB last-level
    # cache: 1.07 GB per Poisson apply), HIP events on the stream it runs on
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wv = torch.empty_like(b0)
    ooc = {}
    for label, h2v, bpp in (("poisson", 0.0, 64), ("helmholtz", 10.0, 72)):
        for _ in range(3):
            s.ax(b0, wv, h1=1.0, h2=h2v)
        ev0.record(stream)
        for _ in range(10):
            s.ax(b0, wv, h1=1.0, h2=h2v)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_a = ev0.elapsed_time(ev1) / 10
        gbs = bpp * s.n_local / (ms_a * 1e-3) / 1e9
        ooc[label] = {"ms": round(ms_a, 4), "algorithmic_bytes": bpp * s.n_local,
                      "achieved_GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    # three Poisson fields through one batched call on the same mesh (G read
    # once per element; beyond the Infinity Cache, so G comes from HBM)
    U3 = torch.stack([b0, torch.flip(b0, (0,)), 0.5 * b0])
    W3 = torch.empty_like(U3)
    for _ in range(3):
        s.ax_multi(U3, W3, h1=1.0, h2=0.0)
    ev0.record(stream)
    for _ in range(10):
        s.ax_multi(U3, W3, h1=1.0, h2=0.0)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_a3 = ev0.elapsed_time(ev1) / 10
    gbs = AX3_BYTES_PER_POINT * s.n_local / (ms_a3 * 1e-3) / 1e9
    ooc["poisson_three_fields"] = {
        "call": "sem_ax_multi, 3 FP64 fields", "ms": round(ms_a3, 4),
        "speedup_vs_three_sem_ax": round(3 * ooc["poisson"]["ms"] / ms_a3, 3),
        "algorithmic_bytes": AX3_BYTES_PER_POINT * s.n_local,
        "achieved_GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    del U3, W3
    # dL/dk (sem_grad_k, the adjoint's coefficient gradient) on the same mesh:
    # u, lam and six G read, gk written, 72 B per local point
    lam = torch.flip(b0, (0,))
    for _ in range(3):
        s.grad_k(b0, lam, h1=1.0, out=wv)
    ev0.record(stream)
    for _ in range(10):
        s.grad_k(b0, lam, h1=1.0, out=wv)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_gk = ev0.elapsed_time(ev1) / 10
    gbs = 72 * s.n_local / (ms_gk * 1e-3) / 1e9
    gk_rec = {"call": "sem_grad_k on the 32^3 mesh (dL/dk = -h1 (D lam)^T G (D u) per copy)",
              "ms": round(ms_gk, 4), "algorithmic_bytes": 72 * s.n_local,
              "achieved_GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    del wv, lam
    # every solution's true residual recomputed by the CPU oracle
    oracle_res = {}
    if not args.no_cpu:
        log("[bench] pcg: oracle residuals of the 32^3 solutions")
        orc = OracleResidual(mesh)
        for pre in pres:
            oracle_res[pre] = []
            for r in res[pre]:
                f = inputs.gaussian_per_node(mesh.gid, r["seed"])
                bh = s.gs(B * torch.tensor(f, device="cuda")) * (W > 0)
                oracle_res[pre].append(float(f"{orc.rel(r['x'].cpu().numpy(), bh.cpu().numpy(), 1.0, 10.0):.3e}"))
        for smo, xs_ in schw_x.items():
            schw[smo + "_single"]["oracle_true_rel_res"] = [float(f"{orc.rel(xq, bq, 1.0, 10.0):.3e}")
                                                            for xq, bq in xs_]
        del orc
    # difference between the two solutions (W-weighted, relative)
    diffs = []
    for a, bb in zip(res.get("pmg", []), res.get("jacobi", [])):
        d = float(torch.sqrt(torch.sum(W * (a["x"] - bb["x"]) ** 2) / torch.sum(W * bb["x"] ** 2)))
        diffs.append(d)
    for runs in res.values():
        for r in runs:
            r.pop("x", None)
    inf = s.info()
    s.free()
    out = {"workload": f"{ne}x{ne}x{ne} deformed box, N=7, Helmholtz h1=1 h2=10, "
                       f"{args.pcg_rhs} RHS, true rel. residual 1e-8",
           "n_unique": inf["n_unique"], "n_local": inf["n_local"], "setup_s": round(t_setup, 3)}
    for pre in pres:
        runs = res[pre]
        out[pre] = {"ms_total": round(sum(r["ms"] for r in runs), 3),
                    "ms_per_rhs": [round(r["ms"], 3) for r in runs],
                    "iters": [r["iters"] for r in runs],
                    "true_rel_res": [float(f"{r['true_rel_res']:.3e}") for r in runs],
                    "status": [r["rc"] for r in runs]}
        if pre == "pmg":
            out[pre]["coarse_iters"] = [r["coarse_iters"] for r in runs]
        if pre in first_call:
            out[pre]["first_call_s"] = round(first_call[pre], 3)
        if pre in oracle_res:
            out[pre]["oracle_true_rel_res"] = oracle_res[pre]
        out[pre]["phases_ms_rhs0"] = phases[pre]
    out["ax_out_of_cache"] = ooc
    out["grad_k"] = gk_rec
    for pre, v in lock.items():
        out[pre + "_lockstep"] = v
        v["speedup_vs_independent"] = round(out[pre]["ms_total"] / v["ms_total"], 3)
    if "apply" in schw:
        out["schwarz_apply"] = schw.pop("apply")
    for smo, v in schw.items():
        name = smo.split("_")[0]
        v["smoother"] = f"Chebyshev-accelerated {name.upper()} (FDM local solves), interval [0.25, 1.1] lambda_max"
        if smo.endswith("_single"):
            if "pmg" in out:
                v["speedup_vs_cheby_jacobi_single"] = round(sum(out["pmg"]["ms_per_rhs"]) / sum(v["ms_per_rhs"]), 3)
            out["pmg_" + smo] = v
            continue
        if "pmg_lockstep" in out:
            v["speedup_vs_cheby_jacobi_lockstep"] = round(out["pmg_lockstep"]["ms_total"] / v["ms_total"], 3)
        out["pmg_" + smo + "_lockstep"] = v
    if len(pres) == 2:
        out["speedup_pmg_vs_jacobi"] = round(out["jacobi"]["ms_total"] / out["pmg"]["ms_total"], 3)
        out["rel_diff_pmg_vs_jacobi"] = [float(f"{d:.3e}") for d in diffs]
    if "jacobi" in out:
        out["gdof_per_s_per_iter_jacobi"] = round(
            inf["n_unique"] * sum(out["jacobi"]["iters"]) / (out["jacobi"]["ms_total"] * 1e-3) / 1e9, 3)
    return out


def bench_projection(args, torch, sem_mod, inputs):
    """A sequence of 10 slowly varying loads (inputs.load_sequence, seed 60,
    period 40, eps 1e-3) on the 32^3 deformed Helmholtz box, FCG + FP32 p-MG to 1e-8:
    from zero against projected initial guesses onto up to 8 earlier
    solutions (cleared first)."""
    N, ne, steps = 7, args.pcg_elems, 10
    mesh = sem_mod.box_mesh(ne, ne, ne, N, deform="cyclic", amp=0.05, bc="dirichlet")
    s = sem_mod.Sem(mesh, levels=(7, 3, 1))
    loads = [torch.tensor(f, device="cuda") for f in inputs.load_sequence(mesh.gid, steps, 60, 40.0)]
    kw = dict(tol=1e-8, h1=1.0, h2=10.0, precond="pmg", coarse_tol=args.coarse_tol,
              coarse_maxit=args.coarse_maxit)
    s.solve(s.rhs(loads[0]), **kw)  # preconditioner setup
    out = {"workload": f"{ne}x{ne}x{ne} deformed box, N=7, Helmholtz h1=1 h2=10, sequence of {steps} "
                       "loads f_n = g0 + sin(2 pi n/40) g1 + (n/40)^2 g2 + 1e-3 h_n, p-MG to 1e-8"}
    for label, L in (("from_zero", 0), ("projected_L8", 8)):
        s.proj_reset()
        its, rels, ms = [], [], 0.0
        for f in loads:
            b = s.rhs(f)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, st, rc = s.solve(b, proj_dim=L, **kw)
            torch.cuda.synchronize()
            ms += (time.perf_counter() - t0) * 1e3
            its.append(st["iters"])
            rels.append(float(f"{st['true_rel_res']:.3e}"))
        out[label] = {"ms_total": round(ms, 3), "iters": its, "true_rel_res_max": max(rels)}
    out["speedup"] = round(out["from_zero"]["ms_total"] / out["projected_L8"]["ms_total"], 3)
    s.free()
    return out


def advect_flops(nq, M):
    """Flops of one element and field in the advection kernel (a multiply-add
    counts 2): i-contractions 4 nq^3 M, j-contractions 6 M^2 nq^2, the
    per-point derivatives, integrand and back-interpolation along k
    M^3 (8 nq + 5), back along j 2 nq^2 M^2 and along i 2 nq^3 M."""
    return 6 * nq ** 3 * M + 8 * nq ** 2 * M ** 2 + M ** 3 * (8 * nq + 5)


def bench_advect(args, torch, sem_mod, inputs):
    """Dealiased advection on the 32^3 deformed box, N = 7, on the 11-point
    Gauss rule (the smallest exact for degree 3N): the three velocity
    components advected by the velocity (the hyperbolic substep's operator),
    one sem_advect call for the three fields, timed with HIP events."""
    N, ne = 7, args.pcg_elems
    mesh = sem_mod.box_mesh(ne, ne, ne, N, deform="cyclic", amp=0.05, bc="neumann")
    s = sem_mod.Sem(mesh)
    t0 = time.perf_counter()
    M = s.advect_setup()
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    c = inputs.vortex_velocity(mesh.x.reshape(-1), mesh.y.reshape(-1), mesh.z.reshape(-1))
    C = torch.tensor(c, device="cuda")
    ct = s.advect_velocity(C)
    out = torch.empty_like(C)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        s.advect(ct, C, out)
    ev0.record(stream)
    for _ in range(args.steps):
        s.advect(ct, C, out)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    ev0.record(stream)
    for _ in range(10):
        s.advect_velocity(C, ct)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_vel = ev0.elapsed_time(ev1) / 10
    nq, E = N + 1, s.E
    nbytes = E * (3 * 2 * 8 * nq ** 3 + 3 * 8 * M ** 3)
    flops = E * 3 * advect_flops(nq, M)
    out_h = out.cpu().numpy() if not args.no_cpu else None
    s.free()
    gbs = nbytes / (ms * 1e-3) / 1e9
    tfs = flops / (ms * 1e-3) / 1e12
    cpu = None
    if not args.no_cpu:
        # the oracle on the first 256 elements, one thread: velocity transform
        # and the three fields, scaled to the whole mesh
        from threadpoolctl import threadpool_limits
        from oracle import advect as oadv
        ns = 256
        sl = slice(0, ns * nq ** 3)
        sub = [a.reshape(-1)[sl] for a in (mesh.x, mesh.y, mesh.z)]
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            ctr = oadv.conv_velocity(N, M, *sub, [cd[sl] for cd in c])
            t1 = time.perf_counter()
            for f in range(3):
                oadv.advect(N, M, ctr, c[f][sl])
            t2 = time.perf_counter()
        # the library's result on the same elements against the oracle's
        # (max-norm error relative to the oracle's max per field)
        errs = []
        for f in range(3):
            ref = oadv.advect(N, M, ctr, c[f][sl])
            errs.append(float(np.max(np.abs(out_h[f][sl] - ref)) / np.max(np.abs(ref))))
        cpu = {"kind": "oracle", "cores": 1, "sample": f"first {ns} elements, numpy one thread, scaled by {E // ns}",
               "ms_advect_3_fields_scaled": round((t2 - t1) * 1e3 * E / ns, 1),
               "ms_velocity_transform_scaled": round((t1 - t0) * 1e3 * E / ns, 1),
               "max_rel_err_vs_oracle": [float(f"{e_:.3e}") for e_ in errs]}
    return {"cpu_oracle": cpu, "workload": f"{ne}x{ne}x{ne} deformed box, N=7, Gauss rule M={M} per direction "
                        "(exact for degree 3N), the 3 velocity components advected by the velocity "
                        "(Taylor-Green-type vortex), one sem_advect call",
            "E": E, "M": M, "ms_advect_3_fields": round(ms, 4), "ms_velocity_transform": round(ms_vel, 4),
            "setup_s": round(t_setup, 3),
            "algorithmic_bytes_per_call": nbytes, "flops_per_call": flops,
            "achieved_GBps": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
            "achieved_TFLOPs_fp64": round(tfs, 2), "frac_fp64_vector_peak": round(tfs / FP64_PEAK_TFS, 4),
            "mdof_gauss_points_per_s": round(E * M ** 3 * 3 / (ms * 1e-3) / 1e6, 1)}


def bench_large(args, torch, sem_mod, inputs):
    """64x64x32 elements on [0,2]x[0,2]x[0,1] (cubic elements of side 1/32),
    cyclic perturbation, N=7 (67,108,864 local points), Poisson (h2 = 0),
    homogeneous Dirichlet, f ~ N(0,1) per node (rng(50)); both solvers to a
    relative residual of 1e-8.  Also times the FP64 element operator alone."""
    N = 7
    t0 = time.perf_counter()
    mesh = sem_mod.box_mesh(64, 64, 32, N, L=(2.0, 2.0, 1.0), deform="cyclic", amp=0.05,
                            bc="dirichlet")
    t_mesh = time.perf_counter() - t0
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    t0 = time.perf_counter()
    s = sem_mod.Sem(mesh, levels=(7, 3, 1))
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    free_setup = torch.cuda.mem_get_info()[0]
    f = torch.tensor(inputs.gaussian_per_node(mesh.gid, 50), device="cuda")
    b = s.rhs(f)
    del f
    inf = s.info()
    nL = inf["n_local"]
    # operator alone
    w = torch.empty_like(b)
    for _ in range(3):
        s.ax(b, w)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(10):
        s.ax(b, w)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_ax = ev0.elapsed_time(ev1) / 10
    del w
    out = {"workload": "64x64x32 deformed box on [0,2]^2x[0,1], N=7, Poisson, 1 RHS, "
                       "relative residual 1e-8",
           "n_unique": inf["n_unique"], "n_local": nL, "mesh_s": round(t_mesh, 2),
           "setup_s": round(t_setup, 3), "ms_ax_fp64": round(ms_ax, 4),
           "ax_fp64_GBps": round(AX_BYTES_PER_POINT * nL / (ms_ax * 1e-3) / 1e9, 1)}
    xs = {}
    for pre in ("pmg", "jacobi"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.solve(b, tol=1e-8, precond=pre, maxit=1)  # builds and caches the preconditioner
        torch.cuda.synchronize()
        t_first = time.perf_counter() - t0
        t0 = time.perf_counter()
        x, st, rc = s.solve(b, tol=1e-8, precond=pre, maxit=50000, coarse_tol=args.coarse_tol,
                            coarse_maxit=args.coarse_maxit)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[pre] = {"ms": round(dt * 1e3, 2), "iters": st["iters"],
                    "true_rel_res": float(f"{st['true_rel_res']:.3e}"), "status": rc,
                    "gdof_per_s_per_iter": round(inf["n_unique"] * st["iters"] / dt / 1e9, 3),
                    "first_call_s": round(t_first, 3)}
        if pre == "pmg":
            out[pre]["coarse_iters"] = st["coarse_iters"]
            _, stt, _ = s.solve(b, tol=1e-8, precond=pre, maxit=50000, timers=1,
                                coarse_tol=args.coarse_tol, coarse_maxit=args.coarse_maxit)
            out[pre]["phases_ms"] = {k: round(stt[k], 3) for k in
                                     ("ms_solve", "ms_ax", "ms_gs", "ms_vec", "ms_prec", "ms_coarse")}
        xs[pre] = x.cpu().numpy()
        del x
    torch.cuda.synchronize()
    free_solved = torch.cuda.mem_get_info()[0]
    out["device_memory_GB"] = {
        "handle_after_setup": round((free0 - free_setup) / 1e9, 2),
        "with_rhs_and_solver_workspaces": round((free0 - free_solved) / 1e9, 2),
        "hbm_total": round(torch.cuda.mem_get_info()[1] / 1e9, 1),
        "note": "device free-memory differences around setup and the two solves (library "
                "allocations plus torch's cached tensors)"}
    W, _ = s.weights()
    Wh = W.cpu().numpy()
    dx = xs["pmg"] - xs["jacobi"]
    out["rel_diff_pmg_vs_jacobi"] = float(f"{np.sqrt(np.sum(Wh * dx * dx) / np.sum(Wh * xs['jacobi'] ** 2)):.3e}")
    out["speedup_pmg_vs_jacobi"] = round(out["jacobi"]["ms"] / out["pmg"]["ms"], 3)
    bh = b.cpu().numpy()
    s.free()
    del b, W
    if not args.no_cpu:
        log("[bench] large: oracle residuals of the 64x64x32 solutions")
        orc = OracleResidual(mesh)
        for pre in ("pmg", "jacobi"):
            out[pre]["oracle_true_rel_res"] = float(f"{orc.rel(xs[pre], bh, 1.0, 0.0):.3e}")
        del orc
    return out


def bench_c1(args, torch, sem_mod, inputs, with_cpu):
    """4x4x4 undeformed unit cube, N=7, Poisson, homogeneous Dirichlet,
    f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z); Jacobi-PCG to 1e-10.  A latency
    configuration (2 MB per operator apply)."""
    import math
    mesh = sem_mod.box_mesh(4, 4, 4, 7)
    s = sem_mod.Sem(mesh)
    ue = inputs.sin3(mesh.x, mesh.y, mesh.z).reshape(-1)
    f = torch.tensor(3 * math.pi ** 2 * ue, device="cuda")
    b = s.rhs(f)
    s.solve(b, tol=1e-10)  # warm-up, builds the Jacobi diagonal
    reps = 5
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        x, st, rc = s.solve(b, tol=1e-10)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    err = float(torch.max(torch.abs(x - torch.tensor(ue, device="cuda"))))
    out = {"workload": "4x4x4 undeformed unit cube, N=7, Poisson, Jacobi-PCG to 1e-10",
           "ms": round(ms, 3), "iters": st["iters"], "true_rel_res": float(f"{st['true_rel_res']:.3e}"),
           "max_err_vs_exact": float(f"{err:.3e}"), "status": rc}
    if with_cpu:
        import oracle
        from oracle import solvers
        xi, _ = oracle.gll(7)
        m = inputs.box_mesh(4, 4, 4, xi)
        lv = solvers.Level(7, m.x, m.y, m.z, m.gid, m.dirichlet)
        bo = lv.rhs(3 * math.pi ** 2 * ue)
        t0 = time.perf_counter()
        xo, ito, _ = solvers.pcg_jacobi(lv, bo, tol=1e-10)
        out["cpu_oracle"] = {"ms": round((time.perf_counter() - t0) * 1e3, 1), "iters": ito,
                             "cores": 1, "kind": "oracle"}
        xg = x.cpu().numpy()
        out["rel_err_vs_oracle_solution"] = float(
            f"{np.sqrt(np.sum(lv.W * (xg - xo) ** 2) / np.sum(lv.W * xo ** 2)):.3e}")
    s.free()
    return out


def bench_adjoint(args, torch, sem_mod, inputs):
    """8x8x8 deformed box, N=7: -div(k grad u) = f with k = exp(0.5 g), loss
    1/2 ||u - u_t||_B^2; forward + backward (hand-written adjoint) time, and
    central differences (h = 1e-6) along one seeded N(0,1) direction for f and
    one for k."""
    from paper_2104_05829_amd import SemSolve
    mesh = sem_mod.box_mesh(8, 8, 8, 7, deform="cyclic", amp=0.05)
    s = sem_mod.Sem(mesh)
    g = inputs.fourier_field(mesh.x, mesh.y, mesh.z, 4, 40).reshape(-1)
    kk = torch.tensor(np.exp(0.5 * g), device="cuda")
    ff = torch.tensor(1.0 + inputs.fourier_field(mesh.x, mesh.y, mesh.z, 4, 41).reshape(-1),
                      device="cuda")
    ut = torch.tensor(inputs.sin3(mesh.x, mesh.y, mesh.z).reshape(-1), device="cuda")
    W, _ = s.weights()
    _, B = s.geometry()
    Bbar = s.gs(B.clone())
    opts = dict(tol=1e-13, maxit=20000)

    def loss_of(u):
        d = u - ut
        return 0.5 * torch.sum(W * Bbar * d * d)

    def fwd_bwd():
        f = ff.clone().requires_grad_(True)
        k = kk.clone().requires_grad_(True)
        L = loss_of(SemSolve.apply(f, k, s, opts, False))
        L.backward()
        return L.item(), f.grad, k.grad

    fwd_bwd()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L, gf, gk = fwd_bwd()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3

    def Lval(f, k):
        with torch.no_grad():
            return loss_of(SemSolve.apply(f, k, s, opts, False)).item()

    rng = np.random.default_rng(42)
    h = 1e-6
    d = torch.tensor(rng.standard_normal(ff.numel()), device="cuda")
    dk = torch.tensor(rng.standard_normal(kk.numel()), device="cuda")
    fd_f = (Lval(ff + h * d, kk) - Lval(ff - h * d, kk)) / (2 * h)
    fd_k = (Lval(ff, kk + h * dk) - Lval(ff, kk - h * dk)) / (2 * h)
    an_f, an_k = float(torch.dot(gf, d)), float(torch.dot(gk, dk))
    s.free()
    out = {"workload": "8x8x8 deformed box, N=7, variable-coefficient Poisson, loss 1/2||u-u_t||_B^2",
           "ms_forward_backward": round(ms, 2), "loss": L,
           "fd_rel_discrepancy_f": float(f"{abs(fd_f - an_f) / abs(an_f):.3e}"),
           "fd_rel_discrepancy_k": float(f"{abs(fd_k - an_k) / abs(an_k):.3e}")}
    return out


def cpu_baseline(mesh, seconds):
    """The oracle's Ax + QQ^T on the full 16^3 N=7 mesh, repeated until
    about `seconds` of CPU time: the checked build (single-threaded C, -O2),
    then the all-core timing build (OpenMP over elements, -O3 -march=native;
    its QQ^T, a sort by global pointer and a sequential accumulation, stays on
    one thread).  Returns both per-apply times with their split."""
    import oracle
    xi, _ = oracle.gll(7)
    D = oracle.dhat(7, xi)
    G, B, _ = oracle.geometry(7, mesh.x, mesh.y, mesh.z)
    from paper_2104_05829_amd import inputs
    u = inputs.uniform_lvector(mesh.n_local, 2)
    out = {}
    for label, lib_, budget in (("one_thread", None, seconds), ("all_cores", oracle_timing_lib(), seconds / 2)):
        reps, t_ax, t_gs = 0, 0.0, 0.0
        t0 = time.perf_counter()
        while True:
            ta = time.perf_counter()
            w = oracle.ax(7, D, G, u, _lib=lib_)
            tb = time.perf_counter()
            oracle.qqt(mesh.gid, w)
            tc = time.perf_counter()
            t_ax += tb - ta
            t_gs += tc - tb
            reps += 1
            if time.perf_counter() - t0 >= budget:
                break
        out[label] = {"ms_apply": (time.perf_counter() - t0) * 1e3 / reps, "ms_ax": t_ax * 1e3 / reps,
                      "ms_qqt": t_gs * 1e3 / reps, "reps": reps,
                      "threads": 1 if lib_ is None else lib_.oracle_threads()}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-pcg", action="store_true")
    ap.add_argument("--no-schwarz", action="store_true", help="skip the CHEBY-ASM / CHEBY-RAS solves")
    ap.add_argument("--no-small", action="store_true", help="skip the 4^3 and adjoint records")
    ap.add_argument("--no-advect", action="store_true", help="skip the dealiased advection record")
    ap.add_argument("--pcg-elems", type=int, default=32)
    ap.add_argument("--pcg-rhs", type=int, default=3)
    ap.add_argument("--pcg-precond", choices=("both", "pmg", "jacobi"), default="both")
    ap.add_argument("--coarse-tol", type=float, default=1e-2)
    ap.add_argument("--coarse-maxit", type=int, default=20)
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 64x64x32 Poisson case (PMG-FCG vs Jacobi-PCG to 1e-8)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain elementwise copy of this many MiB (counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2104_05829_amd import inputs
    from paper_2104_05829_amd import sem as sem_mod

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    sem_mod.lib()  # fail loudly if the HIP library is missing

    log("[bench] operator: 16^3 box, N=7, FP64 sem_ax + sem_gs")
    op = bench_operator(args, torch, sem_mod, inputs)
    value = op["nU"] / (op["ms_step"] * 1e-3) / 1e9
    ax_bytes = AX_BYTES_PER_POINT * op["nL"]
    achieved = ax_bytes / (op["ms_ax"] * 1e-3) / 1e9
    traffic = measured_traffic()
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(op["ms_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "16x16x16 hex box, nodes perturbed by the cyclic sin(2pi.)sin(2pi.) map "
                        "(a=0.05), N=7, FP64 sem_ax + sem_gs (Neumann operator QQ^T A_L u, six G), "
                        "seeded uniform[-1,1] L-vector",
            "E": 4096, "N": 7, "n_local": op["nL"], "n_unique": op["nU"],
            "gdof_local_per_s": round(op["nL"] / (op["ms_step"] * 1e-3) / 1e9, 3),
            "ms_ax": round(op["ms_ax"], 5), "ms_gs": round(op["ms_gs"], 5),
            "ms_step_events_median": round(op["ms_step_median"], 5),
            "ms_step_events_mean": round(op["ms_step_mean"], 5),
        },
        "fp32_step": {
            "call": "sem_ax_level + sem_gs_level, level 0 in FP32 (the smoother precision), same mesh",
            "ms_step": round(op["ms_step32"], 5), "ms_ax": round(op["ms_ax32"], 5),
            "gdof_per_s": round(op["nU"] / (op["ms_step32"] * 1e-3) / 1e9, 3),
            "ax_algorithmic_GBps": round(AX32_BYTES_PER_POINT * op["nL"] / (op["ms_ax32"] * 1e-3) / 1e9, 1),
        },
        "stream_copy": {
            "call": "torch copy of 1 GiB FP64 (1 GiB read + 1 GiB written), HIP events",
            "GBps": round(op["copy_gbs"], 1), "frac_hbm_peak": round(op["copy_gbs"] / HBM_PEAK_GBS, 4),
            "ax_frac_of_copy": round(achieved / op["copy_gbs"], 4),
        },
        "ax_three_fields": {
            "call": "sem_ax_multi, 3 FP64 fields, G read once per element",
            "ms": round(op["ms_ax3"], 5),
            "speedup_vs_three_sem_ax": round(3 * op["ms_ax"] / op["ms_ax3"], 3),
            "algorithmic_GBps": round(AX3_BYTES_PER_POINT * op["nL"] / (op["ms_ax3"] * 1e-3) / 1e9, 1),
            "frac_hbm_peak": round(AX3_BYTES_PER_POINT * op["nL"] / (op["ms_ax3"] * 1e-3) / 1e9
                                   / HBM_PEAK_GBS, 4),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "ax_kernel<8,double> (FP64 Poisson element operator)",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else round(traffic / 1e6, 3),
            "traffic_unit": "MB per launch",
            "algorithmic_bytes_per_launch": ax_bytes,
        },
    }
    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.rand(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)  # reads n*8 bytes, writes n*8 bytes
        torch.cuda.synchronize()
        line["copy_probe"] = {"bytes_read": n * 8, "bytes_written": n * 8, "launches": 3}
    if not args.no_cpu:
        log(f"[bench] cpu baseline: oracle Ax + QQ^T, about {args.cpu_seconds} s")
        cb = cpu_baseline(op["mesh"], args.cpu_seconds)
        one, allc = cb["one_thread"], cb["all_cores"]
        line["cpu_baseline"] = {
            "value": round(op["nU"] / (one["ms_apply"] * 1e-3) / 1e9, 6), "unit": "GDOF/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{one['reps']} applies of the oracle's element operator + QQ^T on the full 16^3 N=7 "
                      f"mesh, single-threaded C (-O2), {one['ms_apply']:.1f} ms per apply "
                      f"(Ax {one['ms_ax']:.1f} + QQ^T {one['ms_qqt']:.1f}), host {os.cpu_count()} logical "
                      f"CPUs, {len(os.sched_getaffinity(0))} available",
            "all_cores": {
                "value": round(op["nU"] / (allc["ms_apply"] * 1e-3) / 1e9, 6), "unit": "GDOF/s",
                "cores": allc["threads"], "kind": "oracle",
                "build": "same C source, -O3 -march=native -fopenmp, OpenMP over elements in Ax; "
                         "QQ^T (sort by pointer + accumulation) on one thread",
                "ms_apply": round(allc["ms_apply"], 2), "ms_ax": round(allc["ms_ax"], 2),
                "ms_qqt": round(allc["ms_qqt"], 2), "reps": allc["reps"],
                "ax_speedup_vs_one_thread": round(one["ms_ax"] / allc["ms_ax"], 2)},
        }
    if not args.no_pcg:
        log("[bench] pcg: 32^3 Helmholtz, FCG+FP32 p-MG vs FP64 Jacobi-PCG to 1e-8")
        line["pcg"] = bench_pcg(args, torch, sem_mod, inputs)
    if not args.no_pcg:
        log("[bench] projection: 10-load sequence, p-MG from zero vs projected guesses")
        line["projection"] = bench_projection(args, torch, sem_mod, inputs)
    if not args.no_advect:
        log("[bench] advection: 32^3 deformed box, N=7, M=11, three fields")
        line["advection"] = bench_advect(args, torch, sem_mod, inputs)
    if not args.no_small:
        log("[bench] 4^3 Poisson Jacobi-PCG and 8^3 adjoint")
        line["c1"] = bench_c1(args, torch, sem_mod, inputs, not args.no_cpu)
        line["adjoint"] = bench_adjoint(args, torch, sem_mod, inputs)
    if not args.no_large:
        log("[bench] large: 64x64x32 Poisson, FCG+FP32 p-MG vs FP64 Jacobi-PCG to 1e-8")
        line["pcg_large"] = bench_large(args, torch, sem_mod, inputs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
