#!/usr/bin/env python3
"""Throughput of one IMEX Runge-Kutta step of the FVLBM D2Q9 + k-omega SST on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload delaunay4m]

Workload (default): seeded Delaunay triangulation of a 4:1 rectangle, ~4.0M triangles, point
density graded x3 toward the bottom wall; walls on the long sides, inlet left, outlet right;
Re_H = 3.6e4, inlet u = 0.05, k = 1e-6, omega = 1e-2 (lattice units); dt = 0.9 x the advective
Courant limit; FP32-deviation storage; initial state: a developed wall-bounded stream (1/7-power
profile near the walls, near-wall omega solution).  Synthetic data: the mesh and the uniform initial state
come from the seeded generator (no datasets).  Prints one JSON line on stdout; progress on stderr.

`value` = cells x steps / second / 1e6 (MLUPS) over the timed region, inputs resident in HBM.
`roofline` = the dominant kernel's algorithmic bytes per launch / its mean HIP-event duration.
`cpu_baseline` = the FP64 CPU oracle timed on a bounded sample of the same workload.
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

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
PROFILES = os.path.join(ROOT, "profiles")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# ----------------------------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------------------------
def cached_mesh(key, make):
    """The generated mesh, kept as an .npz under MESH_CACHE[0] (when set) for later runs."""
    from paper_1812_00394_amd import meshgen as mg
    if not MESH_CACHE[0]:
        return make()
    path = os.path.join(MESH_CACHE[0], key + ".npz")
    if os.path.exists(path):
        return mg.load(path)
    mesh = make()
    os.makedirs(MESH_CACHE[0], exist_ok=True)
    mg.save(mesh, path)
    return mesh


MESH_CACHE = [None]


def workload(name):
    from paper_1812_00394_amd import meshgen as mg
    if name == "delaunay4m":
        mesh = cached_mesh("delaunay4m_seed5", lambda: mg.delaunay_rect(n_points=2_000_000, seed=5))
        U, H, Re = 0.05, 1.0, 3.6e4
        flow = dict(nu=U * H / Re, sst=True, group_u=[[0, 0], [U, 0], [0, 0]], group_rho=[1, 1, 1],
                    group_k=[0, 1e-6, 0], group_w=[0, 1e-2, 0])
        init = dict(profile="channel", U=U, H=H, k=1e-6, w=1e-2)
        return mesh, flow, init, 0.9
    if name == "cavity":
        mesh = mg.cavity()
        nu = 0.1 / 1000
        return mesh, dict(nu=nu, dt=30 * nu, group_u=[[0, 0], [0.1, 0]]), dict(u=(0.0, 0.0)), None
    if name == "backstep":
        mesh = mg.backstep()
        U, Re = 0.05, 3.6e4
        nu = U / Re
        flow = dict(nu=nu, dt=60 * 3 * nu, sst=True, group_u=[[0, 0], [U, 0], [0, 0]], group_rho=[1, 1, 1],
                    group_k=[0, 1e-6, 0], group_w=[0, 1e-2, 0])
        return mesh, flow, dict(u=(0.0, 0.0), k=1e-6, w=1e-2), 0.9
    raise SystemExit(f"unknown workload {name}")


def initial_fields(init, xc, nu):
    """Initial velocity, k, omega at the cell centroids xc [n, 2].  'channel': a developed,
    divergence-free wall-bounded stream between walls at y = 0 and y = H, u = U min(1, (d/0.1H)^(1/7))
    with d the distance to the nearer wall, k uniform, omega = max(omega_in, 6 nu / (beta1 d^2))
    (the near-wall omega solution); otherwise uniform."""
    n = len(xc)
    if init.get("profile") == "channel":
        U, H = init["U"], init["H"]
        d = np.minimum(xc[:, 1], H - xc[:, 1])
        u = np.zeros((n, 2))
        u[:, 0] = U * np.minimum(1.0, (np.maximum(d, 0.0) / (0.1 * H)) ** (1 / 7))
        w = np.maximum(init["w"], 6 * nu / (0.075 * np.maximum(d, 1e-12) ** 2))
        return u, np.full(n, init["k"]), w
    u = np.tile(np.asarray(init["u"], float), (n, 1))
    return u, np.full(n, init.get("k", 0.0)), np.full(n, init.get("w", 1.0))


def make_state(F, M, flow, init, precision, dt_frac):
    p = dict(flow)
    if dt_frac is not None:
        p["dt"] = min(p.get("dt", 1e30), dt_frac * M.max_dt())
    n = M.n_cells
    _, xc, _ = M.geometry()
    u, k, w = initial_fields(init, xc, p["nu"])
    kw = dict(k=k, omega=w) if p.get("sst") else {}
    return F.State(M, p, precision=precision, rho=np.ones(n), u=u, **kw), p


# Algorithmic (compulsory) bytes per cell of one launch of each kernel: every array the kernel
# must read or write counted once (neighbour gathers counted once).  T = bytes per value of the
# state's arithmetic type (4 FP32-deviation, 8 FP64), which is also the type of the geometry the
# sweeps stream; S = edges per cell; wall distance 8 B (FP64).
#   ring : sweep 1 takes f^(1) from f^n and tau on the fly (no collide1 launch): reads f^n, tau,
#          writes f^(2), Ga1 (28 values); sweep 2 reads f^(2), f^n, tau, Ga1, writes f^(3), Q (46);
#          sweep 3 reads f^(3), Q, writes f^{n+1} and rho, u (30).  With dt <= 16 tau0 stage 2
#          recovers Ga1 from f^(2), f^n and tau: 9 values fewer in sweeps 1 and 2
#   tiled: collide1 writes f^(1) (19 values with f^n and tau); sweep 1 reads f^(1) as well (37)
#   split: as tiled, plus the 16 gradient planes each sweep reads back (grad writes them)
def kernel_bytes(T, S, variant="ring", recover=False):
    # ring kernels, triangles: per edge the int16 slot code and the neighbour-centroid offset q
    # (2 values), per cell the vertex offsets from the centroid (2 vertices in FP32, 3 in FP64);
    # normals, midpoints and area are formed from them, and in FP64 the LSQ coefficients too, while
    # FP32 reads the host's LSQ coefficients (2 values per edge).  Other meshes: per edge the slot
    # code and normal, midpoint and neighbour offsets (6 values), per cell 1/area, and the inverse
    # LSQ matrix (FP64) or the LSQ coefficients (FP32, 2 per edge).  The first-boundary-edge index is
    # read by boundary cells only.  Split kernels: both int32 ids and 8 edge values per edge.
    if variant == "ring" and S == 3:
        geo = 2 * S + 2 * T * S + (4 * T + 2 * T * S if T == 4 else 6 * T)
    elif variant == "ring":
        geo = 2 * S + 6 * T * S + T + (2 * T * S if T == 4 else 3 * T)
    else:
        geo = 24 + 8 * T * S + T
    extra = 16 * T if variant == "split" else 0
    return {
        # ring SST (one launch): reads rho, u, v, k, omega, writes k, omega, nu_t, tau (9 values)
        "sst": 9 * T + geo + 8,
        "sst_a": 15 * T + 16 + 2 * T * S + 8,
        "sst_b": 19 * T + 16 + 6 * T * S + T + 8,
        "collide1": 19 * T,
        "grad": 25 * T + 16 + 2 * T * S,
        # recover: stage 2 recovers Ga1 from f^(2) (dt <= 16 tau0), stage 1 does not store it
        "sweep1": ((28 if variant == "ring" else 37) - (9 if recover else 0)) * T + geo + extra,
        "sweep2": (46 - (9 if recover else 0)) * T + geo + extra,
        "sweep3": 30 * T + geo + extra,
        # implicit SST variant, one Jacobi sweep launch: S int32 neighbour ids and 2 couplings per
        # edge slot, R' of k and omega, the previous increments (gathers counted once), the new
        # ones; the finishing sweep reads k^n, omega^n, the strain rate and the wall distance and
        # writes k, omega, nu_t, tau instead of increments
        "sst_jacobi": (4 + 2 * T) * S + 6 * T,
        "sst_jacobi_fin": (4 + 2 * T) * S + 4 * T + 3 * T + 8 + 4 * T,
    }


# Compulsory bytes per cell of a whole step for the method itself (independent of how it is split
# into kernels): f-state traffic of the three stage sweeps (81 values), the SST coupling (14
# values), and the mesh data of four sweeps (3 LBM + 1 SST) held in the same type: area, centroid,
# LSQ coefficients (2 per edge), shared edge normals and midpoints (S/2 edges x 4 values), neighbour
# and edge ids (4 B each per edge); plus the FP64 wall distance.
def step_bytes(T, S):
    geo = T * (1 + 2 + 2 * S + S / 2 * 4) + 4 * S + 4 * S
    return (81 + 14) * T + 4 * geo + 8


# The whole-step model with FP64 geometry: the same 95 state values, with the geometry of four
# sweeps priced in FP64 (area, centroid, neighbour and face ids, LSQ coefficients, 1.5 faces of
# normal and midpoint per triangle: 144 B per sweep) plus the wall distance: 584 B per triangle.
def fp64_geometry_step_bytes(T):
    return 95 * T + 584


# The method's compulsory bytes per cell of each launch with the geometry priced in FP64 (the whole
# step sums to fp64_geometry_step_bytes), on triangle meshes with SST: the state values each sweep
# must read or write in the state's type T, plus 144 B of FP64 triangle geometry per sweep (the SST
# sweep also the wall distance, 8 B).
#   sst    reads rho, u, k, omega, writes k, omega, tau: 8 values
#   sweep1 reads f^n, tau, writes f^(2): 19 values
#   sweep2 reads f^(2), f^n, tau, writes f^(3), Q: 37 values
#   sweep3 reads f^(3), Q, tau, writes f^{n+1}, rho, u: 31 values
def compulsory_kernel_bytes(T):
    return {"sst": 8 * T + 152, "sweep1": 19 * T + 144, "sweep2": 37 * T + 144, "sweep3": 31 * T + 144}


# cell renumbering of every mesh the benchmark builds (the --order option)
ORDER = ["tiles"]


# the sources of the forward kernels the PMC summaries measure (their launch code in fvlbm.hip sets
# only grid and LDS sizes)
FORWARD_SOURCES = ("dual.h", "internal.h", "kernels.h", "lattice.h")


def source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1812_00394_amd", "csrc")
    for name in FORWARD_SOURCES:
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload_name, precision):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if it was taken on the
    current kernel sources; else None."""
    path = os.path.join(PROFILES, f"{kernel}_{workload_name}_{precision}_pmc.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def time_steps(F, st, steps, warmup, stream, kernel_timing=True):
    import torch
    st.step(warmup)
    torch.cuda.synchronize()
    if kernel_timing:
        st.timing(True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    t0 = time.perf_counter()
    st.step(steps)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop)
    kt = st.timing_read() if kernel_timing else None
    if kernel_timing:
        st.timing(False)
    return ms, wall, kt


def cpu_sample(mesh_sample_points):
    """The oracle on a bounded sample of the workload: the same graded-Delaunay generator at
    mesh_sample_points points (about 2 % of the benchmark's cells), same flow and Courant fraction,
    the developed-stream initial state."""
    from oracle import fvlbm_oracle as O
    from paper_1812_00394_amd import meshgen as mg
    m = mg.delaunay_rect(n_points=mesh_sample_points, seed=5)
    U, H, Re = 0.05, 1.0, 3.6e4
    nu = U * H / Re
    orc = O.Oracle(m, O.default_params(nu=nu, dt=1.0, sst=True, group_u=[[0, 0], [U, 0], [0, 0]],
                                       group_rho=[1, 1, 1], group_k=[0, 1e-6, 0], group_w=[0, 1e-2, 0]))
    # same Courant fraction as the GPU run
    G = orc.g
    en = np.maximum(O.EX[:, None] * G.nl[:, 0] + O.EY[:, None] * G.nl[:, 1], 0.0)
    out = np.stack([np.bincount(G.cell, weights=en[a], minlength=G.n) for a in range(9)])
    orc.p["dt"] = 0.9 / (out / G.area).max()
    n = G.n
    u, k0, w0 = initial_fields(dict(profile="channel", U=U, H=H, k=1e-6, w=1e-2), G.xc, nu)
    f, k, w = orc.init_state(np.ones(n), u[:, 0], u[:, 1], k0, w0)
    return orc, f, k, w


def cpu_baseline(mesh_sample_points, steps, repeats=3):
    """The FP64 oracle (plain numpy, one thread) stepping the bounded sample `steps` IMEX steps,
    `repeats` times: cells, steps and the seconds of each run."""
    from threadpoolctl import threadpool_limits
    orc, f, k, w = cpu_sample(mesh_sample_points)
    times = []
    with threadpool_limits(limits=1):
        for _ in range(repeats):
            t0 = time.perf_counter()
            orc.run(f, k, w, steps)
            times.append(time.perf_counter() - t0)
    return orc.g.n, steps, times


def _cpu_all_cores_leg(points, steps, barrier, results):
    from threadpoolctl import threadpool_limits
    orc, f, k, w = cpu_sample(points)
    with threadpool_limits(limits=1):
        barrier.wait()
        t0 = time.perf_counter()
        orc.run(f, k, w, steps)
        results.put((orc.g.n, steps, time.perf_counter() - t0))


def cpu_all_cores(mesh_sample_points, steps, procs):
    """The same oracle run in `procs` processes at once, one thread each, each on its own copy of
    the sample (the oracle has no parallel code of its own): aggregate cell updates per second over
    the slowest process's run.  Started before this process touches the GPU (the workers are new
    interpreters)."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    barrier, results = ctx.Barrier(procs), ctx.Queue()
    ps = [ctx.Process(target=_cpu_all_cores_leg, args=(mesh_sample_points, steps, barrier, results)) for _ in range(procs)]
    for p in ps:
        p.start()
    out = [results.get(timeout=600) for _ in ps]
    for p in ps:
        p.join()
    return out


def cpu_cavity_run():
    """The oracle's whole run of the 4,608-cell cavity (Re 1000, dt = 10 tau0, 500 steps, FP64, one
    thread)."""
    from oracle import fvlbm_oracle as O
    from paper_1812_00394_amd import meshgen as mg
    from threadpoolctl import threadpool_limits
    m = mg.cavity()
    nu = 0.1 / 1000
    orc = O.Oracle(m, O.default_params(nu=nu, dt=10 * 3 * nu, group_u=[[0, 0], [0.1, 0]]))
    n = orc.g.n
    f, _, _ = orc.init_state(np.ones(n), np.zeros(n), np.zeros(n))
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        orc.run(f, None, None, 500)
        dt = time.perf_counter() - t0
    return n, 500, dt


def imex_vs_explicit(F, M_big, flow_big, init_big, dt_frac_big):
    """Per-step cost of the IMEX scheme against the explicit scheme it is compared with (forward
    Euler, dt < 2 tau; per-step cost does not depend on dt): on the 4,608-cell cavity (laminar,
    FP64, launch-bound) and on the benchmark mesh (SST, FP32-dev)."""
    import torch
    from paper_1812_00394_amd import meshgen as mg

    def timed(fn, steps):
        fn(3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn(steps)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps * 1e3

    out = {}
    cav = F.Mesh(mg.cavity(), order=ORDER[0])
    nu = 0.1 / 1000
    n = cav.n_cells
    for name, dt in (("imex", 10 * 3 * nu), ("explicit", 3 * nu)):
        st = F.State(cav, dict(nu=nu, dt=dt, group_u=[[0, 0], [0.1, 0]]), precision="fp64", rho=np.ones(n),
                     u=np.zeros((n, 2)))
        out.setdefault("cavity_4608_fp64", {})[name + "_ms"] = round(timed(st.step if name == "imex" else st.step_explicit, 300), 4)
        del st
    for name in ("imex", "explicit"):
        if name == "imex":
            st, p = make_state(F, M_big, flow_big, init_big, "fp32dev", dt_frac_big)
        else:   # a stable step for the explicit scheme: dt = tau0
            st, p = make_state(F, M_big, dict(flow_big, dt=3 * flow_big["nu"]), init_big, "fp32dev", None)
        fn = st.step if name == "imex" else st.step_explicit
        out.setdefault("delaunay4m_fp32dev", {})[name + "_ms"] = round(timed(fn, 50), 4)
        del st
    for v in out.values():
        v["ratio"] = round(v["imex_ms"] / v["explicit_ms"], 3)
    log(f"IMEX / explicit per step: {out}")
    return out


def backstep_run(F, stream, warmup, steps=2000, adj_steps=400, ckpt=20):
    """The backward-facing step (about 123k hybrid cells, SST, 34 tau0): forward MLUPS in FP32-dev and
    FP64 over `steps` steps, and the adjoint of `adj_steps` recorded steps with a checkpoint every
    `ckpt` steps in both precisions, against the forward time of the same steps."""
    import torch
    mesh, flow, init, dt_frac = workload("backstep")
    M = F.Mesh(mesh, order=ORDER[0])
    n = M.n_cells
    out = {"cells": n, "steps": steps}
    for prec in ("fp32dev", "fp64"):
        st, p = make_state(F, M, flow, init, prec, dt_frac)
        ms, _, kt = time_steps(F, st, steps, warmup, stream, kernel_timing=False)
        if not np.all(np.isfinite(st.moments()["totals"])):
            raise SystemExit(f"backstep {prec}: non-finite state after the timed steps")
        del st
        sta, _ = make_state(F, M, flow, init, prec, dt_frac)
        sta.step(warmup)
        sta.record(adj_steps, ckpt_every=ckpt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sta.adjoint(1, [1.0, 0.0, 0.0])
        torch.cuda.synchronize()
        t_adj = time.perf_counter() - t0
        t_fwd = ms / steps * 1e-3 * adj_steps
        del sta
        out[prec] = {"ms_per_step": round(ms / steps, 4), "mlups": round(n * steps / (ms * 1e-3) / 1e6, 1),
                     "adjoint": {"steps": adj_steps, "ckpt_every": ckpt, "adjoint_s": round(t_adj, 4),
                                 "ratio": round(t_adj / t_fwd, 3)}}
        log(f"backstep {prec}: {ms / steps:.4f} ms/step, adjoint/forward {t_adj / t_fwd:.2f}")
    out["dt_over_tau0"] = round(p["dt"] / (3 * p["nu"]), 2)
    return out


def sweep_variants(F, M, flow, init, dt_frac, stream, args):
    """The step with each sweep variant on the benchmark mesh, both precisions: the ring-tiled cell
    loop the library chooses, the two-kernel cell loop (gradient planes in HBM, then one thread per
    cell) and the edge loop with atomics (gradient planes in HBM, one thread per interior edge adding
    its flux to both cells, then one thread per cell for boundary edges and the stage epilogue).
    Per step and per kernel (HIP events)."""
    out = {}
    steps = max(20, args.steps // 4)
    for prec in ("fp32dev", "fp64"):
        for variant in ("ring", "split", "face"):
            os.environ["FVLBM_SWEEP"] = variant
            try:
                st, _ = make_state(F, M, flow, init, prec, dt_frac)
            finally:
                del os.environ["FVLBM_SWEEP"]
            ms, _, _ = time_steps(F, st, steps, args.warmup, stream, kernel_timing=False)
            _, _, kt = time_steps(F, st, steps, 0, stream, kernel_timing=True)
            if not np.all(np.isfinite(st.moments()["totals"])):
                raise SystemExit(f"sweep variant {variant} {prec}: non-finite state")
            out.setdefault(prec, {})[variant] = {
                "ms_per_step": round(ms / steps, 4),
                "kernels_ms": {k: round(v[0] / v[1], 5) for k, v in kt.items() if v[1]},
                "launches_per_step": {k: v[1] / steps for k, v in kt.items() if v[1]}}
            log(f"sweep variant {variant} {prec}: {ms / steps:.3f} ms/step")
            del st
    return out


def airfoil_run(F, steps, adj_steps=200, ckpt=20):
    """The airfoil workload: 512 x 384 O-mesh (196,608 quads) around the sharp-trailing-edge 12 %
    section, Re 6e6 on the chord, 10 degrees incidence, u_inf = 0.05, dt = 0.9 of the advective
    Courant limit, developed near-wall start, face-value limiter on; lift and drag after `steps`
    steps in FP32-dev and FP64, the throughput of both, and the time of the lift coefficient's
    adjoint over `adj_steps` recorded steps."""
    import torch
    from paper_1812_00394_amd import meshgen as mg
    M = F.Mesh(mg.naca_omesh(), order=ORDER[0])
    n = M.n_cells
    _, _, wd = M.geometry()
    U, c, Re, alpha = 0.05, 1.0, 6e6, np.deg2rad(10.0)
    nu = U * c / Re
    kinf, winf = 1e-3 * U * U / Re, 5 * U / c
    p = dict(nu=nu, dt=min(180 * 3 * nu, 0.9 * M.max_dt()), sst=True, theta=alpha, limiter=1,
             group_u=[[0, 0], [U, 0]], group_rho=[1, 1], group_k=[0, kinf], group_w=[0, winf])
    fac = np.minimum(1.0, (wd / 0.01) ** (1 / 7))
    u0 = np.stack([U * np.cos(alpha) * fac, U * np.sin(alpha) * fac], axis=1)
    w0 = np.maximum(winf, 6 * nu / (0.075 * wd ** 2))
    # a start-up transient, not converged coefficients: the free stream moves U steps dt / c chords
    out = {"cells": n, "steps": steps, "dt_over_tau0": round(p["dt"] / (3 * nu), 2), "limiter": 1,
           "freestream_chords_travelled": round(U * steps * p["dt"] / c, 6),
           "note": "start-up transient from the developed near-wall start, not converged coefficients"}
    for prec in ("fp32dev", "fp64"):
        st = F.State(M, p, precision=prec, rho=np.ones(n), u=u0, k=np.full(n, kinf), omega=w0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        cl, cd = st.lift_drag(1, U, c)
        if not (np.isfinite(cl) and np.isfinite(cd) and np.all(np.isfinite(st.moments()["totals"]))):
            raise SystemExit(f"airfoil {prec}: non-finite state after {steps} steps")
        out[prec] = {"cl": cl, "cd": cd, "mlups": round(n * steps / dt / 1e6, 1)}
        del st
        if adj_steps > 0:
            # the lift coefficient's gradient over adj_steps recorded steps (through the limiter's
            # recorded clip states), against the forward time of the same steps
            st = F.State(M, p, precision=prec, rho=np.ones(n), u=u0, k=np.full(n, kinf), omega=w0)
            st.record(adj_steps, ckpt_every=ckpt)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g, _ = st.adjoint_lift_drag(1, U, c, [1.0, 0.0])
            torch.cuda.synchronize()
            ta = time.perf_counter() - t0
            tf = dt * adj_steps / steps
            out[prec]["adjoint"] = {"steps": adj_steps, "ckpt_every": ckpt, "functional": "lift coefficient",
                                    "adjoint_s": round(ta, 4), "ratio": round(ta / tf, 3),
                                    "gradient": [float(x) for x in g]}
            del st
    out["rel_diff_cl"] = abs(out["fp32dev"]["cl"] - out["fp64"]["cl"]) / abs(out["fp64"]["cl"])
    out["rel_diff_cd"] = abs(out["fp32dev"]["cd"] - out["fp64"]["cd"]) / abs(out["fp64"]["cd"])
    log(f"airfoil {steps} steps: Cl {out['fp64']['cl']:.6g} / {out['fp32dev']['cl']:.6g}, "
        f"Cd {out['fp64']['cd']:.6g} / {out['fp32dev']['cd']:.6g} (FP64 / FP32-dev)")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=int(os.environ.get("WORLD_SIZE", "1")))
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="delaunay4m")
    ap.add_argument("--precision", default="fp32dev", choices=["fp32dev", "fp64"])
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-geo64", action="store_true", help="skip the FP32 run with FP64 geometry")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-points", type=int, default=40_000)
    ap.add_argument("--cpu-steps", type=int, default=30)
    ap.add_argument("--adjoint-steps", type=int, default=50, help="recorded steps of the adjoint timing (0: skip)")
    ap.add_argument("--ckpt", type=int, default=20, help="checkpoint interval of the adjoint")
    ap.add_argument("--no-explicit", action="store_true", help="skip the IMEX / explicit cost comparison")
    ap.add_argument("--order", default="tiles", choices=["morton", "tiles", "rcm", "none"],
                    help="cell renumbering of the meshes (fvlbm_mesh_create order)")
    ap.add_argument("--no-backstep", action="store_true",
                    help="skip the backward-facing step's forward and adjoint timing")
    ap.add_argument("--airfoil-steps", type=int, default=3000,
                    help="steps of the airfoil run (lift and drag in FP32-dev and FP64; 0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (reference kernel for rocprof byte counters)")
    ap.add_argument("--sweep-variants", action="store_true",
                    help="also time the step with the edge loop with atomics and the two-kernel cell loop")
    ap.add_argument("--mesh-cache", default=None,
                    help="directory where the generated benchmark mesh is kept as .npz for later runs")
    args = ap.parse_args()
    ORDER[0] = args.order
    MESH_CACHE[0] = args.mesh_cache
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU sharding of this "
              "path is a design note, not built", file=sys.stderr)
        sys.exit(2)

    # the CPU baseline first: its all-cores leg starts new interpreters, which a process that has
    # touched the GPU must not do
    cpu = None
    if not args.no_cpu_baseline:
        cn, csteps, ctimes = cpu_baseline(args.cpu_sample_points, args.cpu_steps)
        procs = max(1, min(16, len(os.sched_getaffinity(0))))
        legs = cpu_all_cores(args.cpu_sample_points, args.cpu_steps, procs)
        vn, vsteps, vdt = cpu_cavity_run()
        cmed = float(np.median(ctimes))
        wall = max(dt for _, _, dt in legs)
        cpu = {"value": round(cn * csteps / cmed / 1e6, 4), "unit": "MLUPS", "cores": 1, "kind": "oracle",
               "sample": f"a {cn}-cell mesh from the same graded-Delaunay generator as the benchmark's, same flow, "
                         f"SST, FP64, {csteps} IMEX steps, plain numpy oracle on one host thread, median of "
                         f"{len(ctimes)} runs ({', '.join(f'{t:.2f}' for t in ctimes)} s)",
               "all_cores": {"value": round(sum(c * s_ for c, s_, _ in legs) / wall / 1e6, 4), "unit": "MLUPS",
                             "cores": procs,
                             "sample": f"{procs} processes at once, one thread each, each stepping its own copy "
                                       f"of the sample {csteps} steps; cell updates of all over the slowest run "
                                       f"({wall:.2f} s; one process alone: {cmed:.2f} s)"},
               "cavity_4608_full_run": {"cells": vn, "steps": vsteps, "seconds": round(vdt, 2),
                                        "mlups": round(vn * vsteps / vdt / 1e6, 4)}}
        log(f"cpu oracle: {cpu['value']} MLUPS on {cn} cells (1 thread), {cpu['all_cores']['value']} MLUPS "
            f"on {procs} processes; cavity 500 steps in {vdt:.1f} s")

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_1812_00394_amd import fvlbm as F
    F.lib()

    t0 = time.perf_counter()
    mesh, flow, init, dt_frac = workload(args.workload)
    log(f"mesh {mesh['name']}: {len(mesh['cell_ptr']) - 1} cells generated in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    M = F.Mesh(mesh, order=ORDER[0])
    log(f"library preprocessing {time.perf_counter() - t0:.1f}s")
    n = M.n_cells
    S = float(np.mean(np.diff(mesh["cell_ptr"])))
    stream = torch.cuda.current_stream()

    st, p = make_state(F, M, flow, init, args.precision, dt_frac)
    log(f"{args.precision} state ready; dt = {p['dt']:.4g} = {p['dt'] / (3 * p['nu']):.1f} tau0")
    # the timed region runs without per-kernel events; a second pass of the same length takes the
    # per-kernel HIP-event durations for the roofline
    ms, wall, _ = time_steps(F, st, args.steps, args.warmup, stream, kernel_timing=False)
    ms_ev, _, kt = time_steps(F, st, args.steps, 0, stream, kernel_timing=True)
    log(f"{args.precision}: {ms_ev / args.steps:.3f} ms/step with per-kernel events")
    mlups = n * args.steps / (ms * 1e-3) / 1e6
    log(f"{args.precision}: {ms / args.steps:.3f} ms/step, {mlups:.1f} MLUPS (wall {wall:.3f}s)")
    mo = st.moments()
    if not np.all(np.isfinite(mo["totals"])):
        raise SystemExit("non-finite state after the timed steps")

    T = 4 if args.precision == "fp32dev" else 8
    # the variant the library chose: the ring sweep launches no collide1, the split path its grad
    variant = "split" if kt["grad"][1] else ("tiled" if kt["collide1"][1] else "ring")
    kb = kernel_bytes(T, S, variant, recover=p["dt"] <= 16 * 3 * p["nu"])
    per_kernel = {}
    for name, (tms, cnt) in kt.items():
        if cnt:
            avg = tms / cnt
            per_kernel[name] = dict(ms_avg=round(avg, 5), launches=cnt, share=round(tms / ms_ev, 4),
                                    gbs=round(kb[name] * n / (avg * 1e-3) / 1e9, 1))
    dominant = max(per_kernel, key=lambda k: kt[k][0])
    dk = per_kernel[dominant]
    tri_sst = S == 3 and bool(p.get("sst")) and variant == "ring"
    # algorithmic bytes of the dominant launch: the method's compulsory bytes with FP64 geometry
    # (triangles with SST); the kernels as built move fewer (FP32 geometry, values formed on the fly)
    cb = compulsory_kernel_bytes(T)[dominant] if tri_sst else kb[dominant]
    achieved = cb * n / (dk["ms_avg"] * 1e-3) / 1e9
    achieved_built = kb[dominant] * n / (dk["ms_avg"] * 1e-3) / 1e9
    traffic = measured_traffic(dominant, args.workload, args.precision)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": dominant, "algorithmic_bytes_per_cell": cb, "algorithmic_bytes_per_launch": cb * n,
                "as_built": {"bytes_per_cell": kb[dominant], "achieved": round(achieved_built, 1),
                             "frac": round(achieved_built / HBM_PEAK_GBS, 4)},
                # the counters' HBM bytes over the same duration (the rate the memory delivered)
                "traffic_gbs": round(traffic / (dk["ms_avg"] * 1e-3) / 1e9, 1) if traffic else None}
    sb = fp64_geometry_step_bytes(T) if S == 3 and p.get("sst") else step_bytes(T, S)
    step_gbs = sb * n * args.steps / (ms * 1e-3) / 1e9

    extra = {}
    if not args.no_fp64 and args.precision == "fp32dev":
        st64, _ = make_state(F, M, flow, init, "fp64", dt_frac)
        ms64, _, _ = time_steps(F, st64, max(10, args.steps // 2), args.warmup, stream, kernel_timing=False)
        steps64 = max(10, args.steps // 2)
        mlups64 = n * steps64 / (ms64 * 1e-3) / 1e6
        log(f"fp64: {ms64 / steps64:.3f} ms/step, {mlups64:.1f} MLUPS")
        # same number of steps from the same initial state: FP32-deviation error against FP64
        st32, _ = make_state(F, M, flow, init, "fp32dev", dt_frac)
        st32.step(args.warmup + steps64)
        m32, m64 = st32.moments(), st64.moments()
        U = float(init.get("U", np.abs(init.get("u", (0.1,))).max())) or 0.1
        err_u = float(np.abs(m32["u"] - m64["u"]).max() / U)
        err_rho = float(np.abs(m32["rho"] - m64["rho"]).max())
        extra = {"fp64_mlups": round(mlups64, 1), "fp64_ms_per_step": round(ms64 / steps64, 4),
                 "fp32dev_vs_fp64": {"steps": args.warmup + steps64, "max_du_over_U": err_u,
                                     "max_drho": err_rho}}
        del st32
        if not args.no_geo64 and variant == "ring":
            # the same FP32-deviation step with the geometry streamed in FP64 and the edge data formed
            # in FP64 (precision fp32dev_geo64): its time and its error against the same FP64 run
            stg, _ = make_state(F, M, flow, init, "fp32dev_geo64", dt_frac)
            msg, _, _ = time_steps(F, stg, args.steps, args.warmup, stream, kernel_timing=False)
            _, _, ktg = time_steps(F, stg, 20, 0, stream, kernel_timing=True)
            stg2, _ = make_state(F, M, flow, init, "fp32dev_geo64", dt_frac)
            stg2.step(args.warmup + steps64)
            mg_ = stg2.moments()
            extra["fp32dev_geo64"] = {
                "ms_per_step": round(msg / args.steps, 4), "mlups": round(n * args.steps / (msg * 1e-3) / 1e6, 1),
                "kernels_ms": {k: round(v[0] / v[1], 5) for k, v in ktg.items() if v[1]},
                "vs_fp64": {"steps": args.warmup + steps64,
                            "max_du_over_U": float(np.abs(mg_["u"] - m64["u"]).max() / U),
                            "max_drho": float(np.abs(mg_["rho"] - m64["rho"]).max())}}
            log(f"fp32dev_geo64: {msg / args.steps:.3f} ms/step")
            del stg, stg2
        del st64

    adjoint = None
    if args.adjoint_steps > 0 and p.get("sst"):
        import torch
        # forward with checkpoints, then the reverse run (recompute + transposed kernels), timed apart
        sta, _ = make_state(F, M, flow, init, args.precision, dt_frac)
        sta.step(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sta.record(args.adjoint_steps, ckpt_every=args.ckpt)
        torch.cuda.synchronize()
        t_rec = time.perf_counter() - t0
        t0 = time.perf_counter()
        grad = sta.adjoint(1, [1.0, 0.0, 0.0])
        torch.cuda.synchronize()
        t_adj = time.perf_counter() - t0
        t_fwd = ms / args.steps * 1e-3 * args.adjoint_steps
        # the record pass keeps the tapes of the last two segments (counted from the end of the run)
        nseg = -(-args.adjoint_steps // args.ckpt)
        recomputed = max(0, args.adjoint_steps - 2 * args.ckpt) if nseg > 1 else 0
        adjoint = {"steps": args.adjoint_steps, "ckpt_every": args.ckpt, "steps_recomputed": recomputed,
                   "record_s": round(t_rec, 4),
                   "adjoint_s": round(t_adj, 4), "forward_s": round(t_fwd, 4),
                   "ratio": round(t_adj / t_fwd, 3), "functional": "x-force on the walls",
                   "gradient": [float(x) for x in grad]}
        log(f"adjoint of {args.adjoint_steps} steps: {t_adj:.3f}s vs forward {t_fwd:.3f}s (ratio {t_adj / t_fwd:.2f})")
        del sta
        # the whole tape resident in HBM (one segment, no recompute): the same run, same gradient
        sta, _ = make_state(F, M, flow, init, args.precision, dt_frac)
        sta.step(args.warmup)
        sta.record(args.adjoint_steps, ckpt_every=args.adjoint_steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        grad_r = sta.adjoint(1, [1.0, 0.0, 0.0])
        torch.cuda.synchronize()
        t_res = time.perf_counter() - t0
        adjoint["resident_tape"] = {"ckpt_every": args.adjoint_steps, "adjoint_s": round(t_res, 4),
                                    "ratio": round(t_res / t_fwd, 3),
                                    "workspace_gb": round(sta.adj_workspace.numel() / 1e9, 2),
                                    "gradient_max_rel_diff": float(np.max(np.abs(np.array(grad_r) - np.array(grad)) /
                                                                          np.maximum(np.abs(np.array(grad)), 1e-300)))}
        log(f"adjoint with the whole tape resident ({adjoint['resident_tape']['workspace_gb']} GB): {t_res:.3f}s "
            f"(ratio {t_res / t_fwd:.2f})")
        del sta

    per_stage = None
    if p.get("sst") and not args.no_explicit:
        # the per-stage SST coupling (params.sst = 2): one more SST launch per step
        stp, _ = make_state(F, M, dict(flow, sst_stages=1), init, args.precision, dt_frac)
        ms_p, _, _ = time_steps(F, stp, max(20, args.steps // 4), args.warmup, stream, kernel_timing=False)
        ms_p /= max(20, args.steps // 4)
        per_stage = {"ms_per_step": round(ms_p, 4), "over_once_per_step": round(ms_p / (ms / args.steps), 3)}
        log(f"per-stage SST: {ms_p:.3f} ms/step")
        del stp

    implicit = None
    if p.get("sst") and not args.no_explicit:
        # the implicit SST variant (params.sst_sweeps): the SST launch writes the system, then the
        # Jacobi sweep launches
        sweeps = 4
        sti, _ = make_state(F, M, dict(flow, sst_sweeps=sweeps), init, args.precision, dt_frac)
        nst = max(20, args.steps // 4)
        ms_i, _, _ = time_steps(F, sti, nst, args.warmup, stream, kernel_timing=False)
        _, _, kti = time_steps(F, sti, nst, 0, stream, kernel_timing=True)
        # the library times a solve's sweep launches (sweeps - 1 of them) as one interval
        jac_ms, jac_n = kti["sst_jacobi"]
        solve_ms = jac_ms / jac_n
        jb = n * ((sweeps - 2) * kb["sst_jacobi"] + kb["sst_jacobi_fin"])
        asm_key = "sst" if kti["sst"][1] else "sst_b"
        implicit = {"sst_sweeps": sweeps, "ms_per_step": round(ms_i / nst, 4),
                    "over_point_implicit": round((ms_i / nst) / (ms / args.steps), 3),
                    "system_launch_ms": round(kti[asm_key][0] / kti[asm_key][1], 5),
                    "jacobi_launches_per_solve": sweeps - 1,
                    "jacobi_solve_ms": round(solve_ms, 5),
                    "jacobi_algorithmic_gbs": round(jb / (solve_ms * 1e-3) / 1e9, 1)}
        log(f"implicit SST ({sweeps} sweeps): {ms_i / nst:.3f} ms/step, {sweeps - 1} Jacobi launches "
            f"{solve_ms * 1e3:.1f} us ({implicit['jacobi_algorithmic_gbs']} GB/s)")
        del sti

    variants = sweep_variants(F, M, flow, init, dt_frac, stream, args) if args.sweep_variants else None
    airfoil = airfoil_run(F, args.airfoil_steps) if args.airfoil_steps > 0 else None
    backstep = None if args.no_backstep else backstep_run(F, stream, args.warmup)
    cost_ratio = None if args.no_explicit else imex_vs_explicit(F, M, flow, init, dt_frac)

    if args.copy_calibration:
        x = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()

    out = {
        "metric": "MLUPS per IMEX step (FP64 vs FP32-dev) at stated err; adjoint/forward ratio",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32dev" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {n} cells, D2Q9{' + k-omega SST' if p.get('sst') else ''}, "
                               f"{args.precision}, dt {p['dt']:.3g} ({p['dt'] / (3 * p['nu']):.0f} tau0)",
                   "cells": n, "precision": args.precision, "sst": bool(p.get("sst")), "order": args.order},
        "roofline": roofline,
        # the whole step on the method's compulsory bytes (FP64 geometry: 964 B per triangle with SST
        # in FP32-dev, 1,344 B in FP64), and what the kernels as built move
        "step_roofline": {"bytes_per_cell": round(sb, 1), "achieved_gbs": round(step_gbs, 1),
                          "frac": round(step_gbs / HBM_PEAK_GBS, 4),
                          "as_built_bytes_per_cell": sum(kb[k] for k in per_kernel),
                          "as_built_frac": round(sum(kb[k] for k in per_kernel) * n * args.steps / (ms * 1e-3) / 1e9
                                                 / HBM_PEAK_GBS, 4)},
        "kernels": per_kernel,
        "adjoint_forward_ratio": adjoint["ratio"] if adjoint else None,
        "adjoint": adjoint,
        "airfoil_lift_drag": airfoil,
        "backstep": backstep,
        "imex_over_explicit_per_step": cost_ratio,
        "sst_per_stage": per_stage,
        "sst_implicit": implicit,
        "sweep_variants": variants,
        "cpu_baseline": cpu,
        "kernel_source_sha256": source_hash(),
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
