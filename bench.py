"""Benchmark: BBWADG LSRK4 steps on one MI355X.

Workload (the paper's method at the configuration the headline metric is quoted on):
unit cube, 32^3 cells x 6 Kuhn tetrahedra = 196,608 affine tets, N = 5, M = 2, FP64,
c^2 = 1 + 8 seeded Gaussian bumps (amplitude U[-0.4, 0.4], width 0.1, seed 0) projected to
P^2 per element, Gaussian pressure pulse (width 0.05) at the centre, p = 0 walls,
dt from CFL 0.5. Synthetic, seeded inputs; nothing is read from disk.

One step = one full low-storage RK4 step (five fused stage kernels: volume, surface/lift,
WADG multiply + projection and the RK update), inputs resident in HBM. The timed region is
`steps` back-to-back steps on torch's current stream, bracketed by device synchronisation.

Printed: one JSON line with the FP64 throughput in GDOF-updates/s (K Np 4 steps / time),
the roofline of the stage kernel (algorithmic bytes / measured launch time vs 8 TB/s),
an FP32 leg of the same workload with its per-field L2 difference from FP64, and the CPU
oracle timed on a bounded sample.
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
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CELLS, N, M = 32, 5, 2
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stage_kernel_cube196k_N5_M2_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1808_08645_amd", "csrc", "stage_kernel.hpp")


def dimp(n):
    return (n + 1) * (n + 2) * (n + 3) // 6


# Connectivity bytes per element: four int32 neighbour ids (4 k' + f', or -1 on a wall).
CONN_BYTES = 16


def algorithmic_bytes_per_element(n, m, word):
    """One fused stage reads q and res and writes q and res (16 Np words), reads the c^2
    coefficients (Mp words), the geometry record (25 words: G, Fscale and n per face) and
    the 4 neighbour ids (CONN_BYTES = 16: the ids are int32; a layout with 8-byte ids would
    count 32)."""
    return (16 * dimp(n) + dimp(m) + 25) * word + CONN_BYTES


def kernel_source_hash():
    """sha256 (16 hex digits) of the stage kernel source with comments and blank space
    removed, so that counters stay attached to the code they were taken on."""
    import re
    with open(KERNEL_SRC) as fh:
        src = fh.read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    src = " ".join(src.split())
    return hashlib.sha256(src.encode()).hexdigest()[:16]


def measured_traffic(dtype="f64"):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were taken on
    the current kernel source; otherwise None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_code_sha256_16") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch_" + dtype)


def setup(dtype):
    import paper_1808_08645_amd as bb
    from workloads import c2_gaussian_bumps, ic_gaussian_pulse, kuhn_cube_mesh

    xyz, etov = kuhn_cube_mesh(CELLS)
    s = bb.Solver(xyz, etov, N, M, dtype=dtype)
    s.project_c2(c2_gaussian_bumps(0))
    zero = lambda x, y, z: 0.0 * x  # noqa: E731
    q0 = s.initial_state([ic_gaussian_pulse, zero, zero, zero])
    return s, q0


def run_leg(s, q0, dt, steps, warmup, chunks=1):
    """Advance q0 by warmup untimed steps, then time exactly `steps` steps as one region on
    the launch stream. With chunks > 1 the region is split into that many back-to-back
    parts by events on the same stream (no synchronisation in between), whose per-step times
    are returned too (their median is robust to one slow part)."""
    import torch
    q = s.to_device(q0)
    res = torch.zeros_like(q)
    if warmup:
        s.step(q, res, dt, warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    chunks = max(1, min(chunks, steps))
    sizes = [steps // chunks + (1 if i < steps % chunks else 0) for i in range(chunks)]
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(chunks + 1)]
    t0 = time.perf_counter()
    evs[0].record(stream)
    for i, n in enumerate(sizes):
        s.step(q, res, dt, n)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = evs[0].elapsed_time(evs[-1])
    per_step = [evs[i].elapsed_time(evs[i + 1]) / n for i, n in enumerate(sizes)]
    # An odd total stage count ends with one state copy; time it alone to take it out.
    copy_ms = 0.0
    if (5 * steps) % 2 == 1:
        tmp = torch.empty_like(q)
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        tmp.copy_(q)
        c1.record(stream)
        torch.cuda.synchronize()
        copy_ms = c0.elapsed_time(c1)
    if chunks > 1:
        return q, ms, wall, copy_ms, per_step
    return q, ms, wall, copy_ms


def copy_bandwidth(mib=1024, reps=5):
    """A plain device-to-device copy of `mib` MiB (torch's copy kernel), timed with events on
    the current stream, median of `reps`: bytes read + written over time. This is the
    streaming bandwidth a kernel can reach on this GPU, next to the 8 TB/s nominal peak."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        dst.copy_(src)
        e1.record(st)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = sorted(ts)[len(ts) // 2]
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes": 2 * n * 8, "ms": ms, "gbs": 2 * n * 8 / (ms * 1e-3) / 1e9, "reps": reps}


def c1_entry():
    """The small configuration: 4^3 x 6 = 384 tets, N=3, M=1, c^2 = 1 + 0.5 sin sin sin
    projected to P^1, p0 = cos cos cos, p = 0 walls, 10 LSRK4 steps at CFL 0.5, in FP64 and
    FP32 (median of 5 runs of the 10 steps). Its 245 KB of state sit in cache, so the rate
    is launch-bound and has no roofline meaning."""
    import torch

    import paper_1808_08645_amd as bb
    from workloads import c2_sinusoid, ic_cos_product, kuhn_cube_mesh
    xyz, etov = kuhn_cube_mesh(4)
    zero = lambda x, y, z: 0.0 * x  # noqa: E731
    out = {"workload": "cube384_N3_M1", "elements": len(etov), "steps": 10}
    for dtype in ("f64", "f32"):
        s = bb.Solver(xyz, etov, 3, 1, dtype=dtype)
        s.project_c2(c2_sinusoid)
        q0 = s.initial_state([ic_cos_product, zero, zero, zero])
        dt = s.suggest_dt(0.5)
        ts = []
        for _ in range(6):
            _, ms, _, _ = run_leg(s, q0, dt, 10, 0)
            ts.append(ms)
        ms = sorted(ts[1:])[2]
        out[dtype] = {"ms_per_step": ms / 10, "gdof_updates_per_s": s.K * s.Np * 4 * 10 / (ms * 1e-3) / 1e9}
        s.close()
    torch.cuda.empty_cache()
    return out


def _ring(nbr, seeds, rings):
    sel = set(int(x) for x in seeds)
    front = set(sel)
    for _ in range(rings):
        nxt = {int(v) >> 2 for k in front for v in nbr[k] if v >= 0}
        front = nxt - sel
        sel |= nxt
    return np.array(sorted(sel))


def oracle_parity(s, xyz, etov, q, nsample=24, seed=0):
    """Per-field relative L2 error of the device right-hand side at state q (the benchmark's
    final state) against the oracle, on sampled elements: the oracle evaluates the same
    coefficients and the same c^2_M on the sampled elements and their face neighbours."""
    from oracle import Oracle
    rng = np.random.default_rng(seed)
    K = s.K
    cen = xyz[etov].mean(axis=1)
    near = np.argsort(np.linalg.norm(cen - 0.5, axis=1))[:8]  # where the pulse is
    seeds = np.unique(np.concatenate([near, rng.choice(K, nsample - len(near), replace=False)]))
    r = s.rhs(q).double().cpu().numpy()
    qh = q.double().cpu().numpy()
    sub = _ring(s.geometry()["nbr"], seeds, 1)
    o = Oracle(xyz, etov[sub], s.N, s.M)
    o.set_c2_bernstein(s.get_c2()[sub])
    R = o.rhs(o.from_bernstein(qh[:, sub]))
    pos = np.searchsorted(sub, seeds)
    a = o.bernstein_values_at_quad(r[:, seeds])
    b = o.values_at_quad(R[:, pos])
    wJ = o.mesh.J[pos][:, None] * o.wq[None, :]
    num = np.sum((a - b) ** 2 * wJ, axis=(1, 2))
    den = np.maximum(np.sum(b ** 2 * wJ, axis=(1, 2)), 1e-300)
    return {"rel_l2_per_field": np.sqrt(num / den).tolist(), "elements": int(len(seeds)),
            "what": "right-hand side at the final benchmark state, sampled elements (8 at the pulse, the rest random, seed 0)"}


def cpu_baseline(dt, steps):
    """The oracle (dense quadrature WADG, FP64, NumPy/OpenBLAS) timed on a bounded sample:
    the same workload on 16^3 cells x 6 = 24,576 tets, `steps` LSRK4 steps."""
    from threadpoolctl import threadpool_info

    from oracle import Oracle
    from workloads import c2_gaussian_bumps, ic_gaussian_pulse, kuhn_cube_mesh
    cells = 16
    xyz, etov = kuhn_cube_mesh(cells)
    o = Oracle(xyz, etov, N, M)
    o.set_c2_function(c2_gaussian_bumps(0), project=True)
    zero = lambda x, y, z: 0.0 * x  # noqa: E731
    Q = o.project_initial([ic_gaussian_pulse, zero, zero, zero])
    t0 = time.perf_counter()
    o.step(Q, np.zeros_like(Q), dt, steps)
    t = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info() if p.get("user_api") == "blas"] or [1])
    K = len(etov)
    return {"value": K * dimp(N) * 4 * steps / t / 1e9, "unit": "GDOF-updates/s", "cores": int(threads),
            "kind": "oracle", "seconds": t,
            "sample": f"cube 16^3x6 = {K} tets, N={N}, M={M}, same medium and pulse, {steps} LSRK4 steps, FP64"}


def c3_sweep(steps, warmup, n_list=range(4, 10)):
    """The 196,608-tet mesh at N = 4..9, M = N/2, three-layer medium (c^2 in {1, 2, 4}, seed 1)
    projected to P^M, Gaussian pulse: FP64 and FP32 throughput and per-field FP32-vs-FP64
    relative L2 after warmup + steps LSRK4 steps (both legs share the c^2_M data).

    The P^M projection of the layered medium is not positive everywhere (the exact check
    rejects it by default); the sweep accepts it on purpose and reports, per N, how many
    elements have a c^2_M that is not positive, and the FP64 state norm and energy over the
    run. A row whose norm exceeds twice its start is an unstable run: its FP32-vs-FP64
    difference measures the growth, not the precision."""
    import torch

    import paper_1808_08645_amd as bb
    from workloads import c2_three_layer, ic_gaussian_pulse, kuhn_cube_mesh
    xyz, etov = kuhn_cube_mesh(CELLS)
    out = []
    for n in n_list:
        m = n // 2
        s64 = bb.Solver(xyz, etov, n, m, dtype="f64")
        s64.set_c2_policy(True)
        c2 = s64.project_c2(c2_three_layer(1))
        nonpos, undecided = s64.c2_positivity()
        q0 = np.zeros((4, s64.K, s64.Np))
        q0[0] = s64.project_function(ic_gaussian_pulse, n)
        dt = s64.suggest_dt(0.5)
        q64, ms64, _, copy64 = run_leg(s64, q0, dt, steps, warmup)
        s32 = bb.Solver(xyz, etov, n, m, dtype="f32")
        s32.set_c2_policy(True)
        s32.set_c2(c2)
        q32, ms32, _, copy32 = run_leg(s32, q0, dt, steps, warmup)
        diff = (q32.double() - q64).contiguous()
        rel = np.sqrt(s64.l2norm2(diff) / np.maximum(s64.l2norm2(q64), 1e-300)).tolist()
        dofs = s64.K * s64.Np * 4
        entry = {"N": n, "M": m, "dofs": dofs, "dt": dt, "c2_nonpositive_elements": int(nonpos),
                 "c2_undecided_elements": int(undecided)}
        for tag, ms, cp, word in (("f64", ms64, copy64, 8), ("f32", ms32, copy32, 4)):
            kms = (ms - cp) / (5 * steps)
            entry[tag] = {"gdof_updates_per_s": dofs * steps / (ms * 1e-3) / 1e9, "ms_per_step": ms / steps,
                          "kernel_ms": kms,
                          "alg_frac_hbm": algorithmic_bytes_per_element(n, m, word) * s64.K / (kms * 1e-3) / 1e9
                          / HBM_PEAK_GBS}
        # FP64 norm and energy trace over the same number of steps, in four parts
        q = s64.to_device(q0)
        res = torch.zeros_like(q)
        total = warmup + steps
        trace = [{"step": 0, "norm": float(np.sqrt(s64.l2norm2(q).sum())), "energy": float(s64.energy(q).sum())}]
        done = 0
        for part in range(4):
            k = total * (part + 1) // 4 - done
            s64.step(q, res, dt, k)
            done += k
            trace.append({"step": done, "norm": float(np.sqrt(s64.l2norm2(q).sum())),
                          "energy": float(s64.energy(q).sum())})
        entry["fp64_trace"] = trace
        # With 1 <= c^2 <= 4 an energy-stable run keeps |q(t)|^2 <= 4 * 2E(t) <= 4 * 2E(0) <= 4 |q(0)|^2
        # (E = 1/2 int p^2/c^2 + |u|^2), so a norm above twice the start is growth, not exchange.
        stable = max(t["norm"] for t in trace) <= 2.0 * trace[0]["norm"]
        entry["stable"] = bool(stable)
        entry["fp32_rel_l2_vs_fp64_per_field"] = rel
        if not stable:
            entry["note"] = "the FP64 state norm grows: an unstable run, the FP32-vs-FP64 difference is not a precision figure"
        out.append(entry)
        print(json.dumps({"c3_progress": entry}), file=sys.stderr, flush=True)
        del s64, s32, q64, q32, diff, q, res
        torch.cuda.empty_cache()
    return out


def wadg_compare(n_list, m_list, reps, cells=None, dtypes=("f64", "f32")):
    """Dense quadrature WADG (matrix cores) against the Bernstein update on the 196,608-tet mesh,
    in each precision: times of the fused Bernstein right-hand side, the plain DG right-hand
    side (c^2 = 1, no weight adjustment), and the dense update alone, with c^2_M of the bump
    medium at the points."""
    import torch

    import paper_1808_08645_amd as bb
    from workloads import kuhn_cube_mesh
    xyz, etov = kuhn_cube_mesh(cells or CELLS)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = []
    for dtype in dtypes:
        word = 8 if dtype == "f64" else 4
        for n in n_list:
            # the plain DG right-hand side: the fused kernel with M = 0 and c^2 = 1
            s0 = bb.Solver(xyz, etov, n, 0, dtype=dtype)
            s0.set_c2(np.ones((s0.K, 1)))
            q0 = s0.to_device(np.random.default_rng(5).uniform(-1, 1, (4, s0.K, s0.Np)))
            r0 = torch.empty_like(q0)
            t_dg = timed(lambda: s0.rhs(q0, r0))
            del s0, q0, r0
            for m in m_list:
                if m > n:
                    continue
                s = bb.Solver(xyz, etov, n, m, dtype=dtype)
                s.project_c2(c2_bumps_medium())
                s.dense_set_c2(None)
                q = s.to_device(np.random.default_rng(5).uniform(-1, 1, (4, s.K, s.Np)))
                r = torch.empty_like(q)
                t_bb = timed(lambda: s.rhs(q, r))
                t_dense_rhs = timed(lambda: s.rhs_dense(q, r))
                p0 = q[0].contiguous()
                p1 = torch.empty_like(p0)
                t_dense = timed(lambda: s.dense_update(p0, p1))
                t_bupd = timed(lambda: s.wadg_update(p0, p1))
                e = {"dtype": dtype, "N": n, "M": m, "Np": s.Np, "nq_dense": s.dense_npoints(),
                     "rhs_bernstein_ms": t_bb, "rhs_dense_ms": t_dense_rhs, "dense_update_ms": t_dense,
                     "plain_dg_rhs_ms": t_dg, "bernstein_update_ms": t_bupd, "fused_minus_plain_ms": t_bb - t_dg,
                     "elements": s.K, "bernstein_update_us_per_element": t_bupd * 1e3 / s.K,
                     "dense_update_us_per_element": t_dense * 1e3 / s.K,
                     "bernstein_update_gb_s": (2 * s.Np + s.Mp) * word * s.K / (t_bupd * 1e-3) / 1e9,
                     "dense_update_tflops": 4.0 * s.dense_npoints() * s.Np * s.K / (t_dense * 1e-3) / 1e12,
                     "dense_update_frac_of_mfma_peak": 4.0 * s.dense_npoints() * s.Np * s.K / (t_dense * 1e-3) / 1e12
                     / (78.6 if dtype == "f64" else 157.3)}
                out.append(e)
                print(json.dumps({"wadg_compare_progress": e}), file=sys.stderr, flush=True)
                del s, q, r, p0, p1
                torch.cuda.empty_cache()
    return out


def rates_sweep(n_list, m_list, meshes, T=0.5, cfl=0.5):
    """The 3D manufactured solution of paper Section 6.1 (c^2 = 1 + sin sin sin / 2 projected
    onto P^M, pressure source, p = 0 walls) to time T: L^2 errors of the pressure and of the
    velocity on each Kuhn cube and the observed rates between consecutive meshes, in FP64."""
    import torch

    import paper_1808_08645_amd as bb
    from workloads import c2_sinusoid, kuhn_cube_mesh, manufactured_solution, manufactured_source

    def fields(t):
        return [lambda x, y, z, i=i: manufactured_solution(x, y, z, t)[i] for i in range(4)]

    out = []
    for n in n_list:
        for m in m_list:
            if m > n:
                continue
            errs = []
            for cells in meshes:
                xyz, etov = kuhn_cube_mesh(cells)
                s = bb.Solver(xyz, etov, n, m, dtype="f64")
                s.project_c2(c2_sinusoid)
                s.set_source(manufactured_source(c2_sinusoid), omega=np.pi)
                nsteps = int(np.ceil(T / s.suggest_dt(cfl)))
                q = s.to_device(s.initial_state(fields(0.0)))
                res = torch.zeros_like(q)
                s.step(q, res, T / nsteps, nsteps)
                torch.cuda.synchronize()
                errs.append(s.l2error2(q, fields(T)))
                del s, q, res
            E = np.array(errs)
            ep, eu = np.sqrt(E[:, 0]), np.sqrt(E[:, 1:].sum(1))
            e = {"N": n, "M": m, "cells": list(meshes), "l2_error_p": ep.tolist(), "l2_error_u": eu.tolist(),
                 "rates_p": np.log2(ep[:-1] / ep[1:]).tolist(), "rates_u": np.log2(eu[:-1] / eu[1:]).tolist(),
                 "paper_rate_p": 2 if m == 0 else min(n + 1, m + 3)}
            out.append(e)
            print(json.dumps({"rates_progress": e}), file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
    return out


def adjoint_bench(nsteps=500, ckpt=50, n_fd=20):
    """Misfit gradient on 24^3 x 6 = 82,944 tets, N=4, M=2, rigid walls, 64 receivers on the
    top face, nsteps LSRK4 steps at CFL 0.5, checkpoints every ckpt steps. The observed traces
    come from a seeded target medium (bumps, seed 5); the gradient is taken at the bump medium
    (seed 0). Times the forward run alone and forward + gradient in FP64 and FP32, compares the
    FP32 gradient with the FP64 one, and checks the FP64 gradient against central differences
    of the misfit on n_fd seeded coefficients."""
    import time

    import torch

    import paper_1808_08645_amd as bb
    from workloads import c2_gaussian_bumps, ic_gaussian_pulse, kuhn_cube_mesh, receiver_grid
    xyz, etov = kuhn_cube_mesh(24)
    pulse = lambda x, y, z: ic_gaussian_pulse(x, y, z, centre=(0.5, 0.5, 0.85), width=0.1)  # noqa: E731
    zero = lambda x, y, z: 0.0 * x  # noqa: E731
    out = {"elements": int(etov.shape[0]), "N": 4, "M": 2, "receivers": 64, "steps": nsteps,
           "checkpoint_every": ckpt}
    grads = {}
    for dtype in ("f64", "f32"):
        s = bb.Solver(xyz, etov, 4, 2, dtype=dtype, bc="rigid")
        s.set_receivers(receiver_grid(8, 1.0))
        q0 = s.initial_state([pulse, zero, zero, zero])
        q = s.to_device(q0)
        if dtype == "f64":
            target = s.project_c2(c2_gaussian_bumps(5))
            c = s.project_c2(c2_gaussian_bumps(0))
            dt = s.suggest_dt(0.5)
            s.set_c2(target)
            _, _, data = s.misfit_gradient(q, dt, nsteps, None, gradient=False)
            out["dt"] = dt
        s.set_c2(c)
        s.misfit_gradient(q, dt, 5, data[:5].contiguous(), ckpt)  # warm-up (tables, code objects)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J, _, _ = s.misfit_gradient(q, dt, nsteps, data, ckpt, gradient=False)
        t1 = time.perf_counter()
        J2, g, _ = s.misfit_gradient(q, dt, nsteps, data, ckpt)
        t2 = time.perf_counter()
        grads[dtype] = g.cpu().numpy()
        dofs = s.K * s.Np * 4
        out[dtype] = {"misfit": J, "forward_s": t1 - t0, "forward_and_gradient_s": t2 - t1,
                      "gradient_over_forward": (t2 - t1) / (t1 - t0),
                      "forward_gdof_updates_per_s": dofs * nsteps / (t1 - t0) / 1e9}
        print(json.dumps({"adjoint_progress": {dtype: out[dtype]}}), file=sys.stderr, flush=True)
        if dtype == "f64":
            s64, q64 = s, q
        else:
            del s, q
    g64, g32 = grads["f64"], grads["f32"]
    out["f32_vs_f64_gradient_rel_l2"] = float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64))
    if n_fd <= 0:
        return out
    rng = np.random.default_rng(11)
    big = np.nonzero(np.abs(g64).max(1) > 1e-2 * np.abs(g64).max())[0]
    rel = []
    for k in rng.choice(big, n_fd, replace=False):
        b = int(rng.integers(s64.Mp))
        h = 1e-4 * max(1.0, abs(c[k, b]))
        cp, cm = c.copy(), c.copy()
        cp[k, b] += h
        cm[k, b] -= h
        s64.set_c2(cp)
        jp = s64.misfit_gradient(q64, dt, nsteps, data, ckpt, gradient=False)[0]
        s64.set_c2(cm)
        jm = s64.misfit_gradient(q64, dt, nsteps, data, ckpt, gradient=False)[0]
        fd = (jp - jm) / (2 * h)
        rel.append(abs(fd - g64[k, b]) / np.abs(g64).max())
    s64.set_c2(c)
    out["fd_check"] = {"coefficients": n_fd, "max_abs_diff_over_max_grad": float(max(rel)),
                       "median": float(np.median(rel)), "step": "1e-4 max(1, |c|)"}
    return out


def surrogate_bench(n_models=256, n_train=224, nsteps=400, train_steps=4000, batch=32):
    """Trace surrogate on 16^3 x 6 = 24,576 tets, N=4, M=2 (rigid walls, 64 receivers on the top
    face, Gaussian pulse at (0.5, 0.5, 0.85), nsteps steps at one dt for every medium): BBWADG
    makes the traces of n_models seeded media (FP64), the surrogate trains on n_train of them
    (Adam, cosine learning rate 1e-3 -> 1e-5) and is scored against BBWADG on the rest."""
    import time

    import torch

    import paper_1808_08645_amd as bb
    from paper_1808_08645_amd.surrogate import Surrogate
    from workloads import c2_random_model, grid_centres, ic_gaussian_pulse, kuhn_cube_mesh, receiver_grid
    xyz, etov = kuhn_cube_mesh(16)
    s = bb.Solver(xyz, etov, 4, 2, dtype="f64", bc="rigid")
    s.set_receivers(receiver_grid(8, 1.0))
    pulse = lambda x, y, z: ic_gaussian_pulse(x, y, z, centre=(0.5, 0.5, 0.85), width=0.1)  # noqa: E731
    zero = lambda x, y, z: 0.0 * x  # noqa: E731
    q = s.to_device(s.initial_state([pulse, zero, zero, zero]))
    s.project_c2(lambda x, y, z: 4.0 + 0.0 * x)
    dt = s.suggest_dt(0.5)
    gx, gy, gz = grid_centres(16)
    X = np.zeros((n_models, 16, 16, 16), dtype=np.float32)
    Y = np.zeros((n_models, nsteps * 64), dtype=np.float32)
    t_solver = 0.0
    for i in range(n_models):
        f = c2_random_model(i)
        X[i] = f(gx, gy, gz)
        s.project_c2(f)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, tr = s.misfit_gradient(q, dt, nsteps, None, gradient=False)
        torch.cuda.synchronize()
        t_solver += time.perf_counter() - t0
        Y[i] = tr.cpu().numpy().ravel()
        if i % 64 == 63:
            print(json.dumps({"surrogate_progress": f"{i + 1} media simulated"}), file=sys.stderr, flush=True)
    xin = (X - 2.5) / 1.5
    sigma = float(Y[:n_train].std())
    yt = Y / sigma
    sur = Surrogate(nsteps * 64, batch, seed=1)
    xd = torch.tensor(xin, device="cuda")
    yd = torch.tensor(yt, device="cuda")
    rng = np.random.default_rng(2)
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(train_steps):
        idx = torch.tensor(rng.choice(n_train, batch, replace=False), device="cuda")
        lr = 1e-5 + 0.5 * (1e-3 - 1e-5) * (1 + np.cos(np.pi * k / train_steps))
        losses.append(sur.train_step(xd[idx], yd[idx], lr))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    # score on the held-out media
    test = np.arange(n_train, n_models)
    preds = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a in range(0, len(test), batch):
        preds.append(sur.forward(xd[test[a:a + batch]]))
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    P = torch.cat(preds).cpu().numpy() * sigma
    T = Y[test]
    err = np.linalg.norm(P - T, axis=1) / np.linalg.norm(T, axis=1)
    mean_pred = Y[:n_train].mean(0)
    err_mean = np.linalg.norm(mean_pred[None] - T, axis=1) / np.linalg.norm(T, axis=1)
    Ptr = []
    for a in range(0, n_train, batch):
        Ptr.append(sur.forward(xd[a:min(n_train, a + batch)]))
    Ptr = torch.cat(Ptr).cpu().numpy() * sigma
    err_train = np.linalg.norm(Ptr - Y[:n_train], axis=1) / np.linalg.norm(Y[:n_train], axis=1)
    return {"elements": int(etov.shape[0]), "N": 4, "M": 2, "receivers": 64, "steps": nsteps, "dt": dt,
            "media": n_models, "train": n_train, "held_out": int(len(test)), "parameters": sur.num_params,
            "train_steps": train_steps, "batch": batch, "loss_first_last": [losses[0], losses[-1]],
            "held_out_rel_l2": {"mean": float(err.mean()), "median": float(np.median(err)), "max": float(err.max())},
            "train_rel_l2_mean": float(err_train.mean()),
            "mean_trace_predictor_rel_l2_mean": float(err_mean.mean()),
            "accepted_below_0.2": int((err < 0.2).sum()), "fallback_to_bbwadg": int((err >= 0.2).sum()),
            "bbwadg_s_per_medium": t_solver / n_models, "surrogate_s_per_medium": t_inf / len(test),
            "train_s": t_train}


def elastic_bench(reps=20, only=None):
    """Elastic weight-adjusted update (9 fields, isotropic media projected to P^M), N = 2..9,
    M = 1, 2, on the 11^3 x 6 = 7,986-tet mesh (about the size of the paper's 7,854-element timing
    mesh) and on the 196,608-tet mesh: time per launch and per element, FP64 and FP32, next to
    nine dense quadrature updates (the cost of the same update by quadrature WADG); and the
    elastic DG right-hand side, with and without the update, and one 5-stage time step."""
    import torch

    import paper_1808_08645_amd as bb
    from workloads import c2_gaussian_bumps, c2_sinusoid, kuhn_cube_mesh

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = []
    for cells in (11, 32):
        xyz, etov = kuhn_cube_mesh(cells)
        for n in range(2, 10):
            for m in (1, 2):
                if only is not None and (cells, n, m) != only:
                    continue
                e = {"elements": int(etov.shape[0]), "N": n, "M": m}
                for dtype in ("f64", "f32"):
                    s = bb.Solver(xyz, etov, n, m, dtype=dtype)
                    s.elastic_set_media(lambda x, y, z: 1.0 / (1.0 + 0.3 * x), c2_gaussian_bumps(0),
                                        lambda x, y, z: 0.5 * c2_sinusoid(x, y, z))
                    wt = torch.float64 if dtype == "f64" else torch.float32
                    r = torch.randn((9, s.K, s.Np), dtype=wt, device="cuda")
                    o = torch.empty_like(r)
                    ms = timed(lambda: s.elastic_update(r, o))
                    e[dtype] = {"ms": ms, "us_per_element": ms * 1e3 / s.K}
                    # the DG right-hand side before the media: reads the 9 fields and the 9
                    # neighbour face traces, writes 9 fields (algorithmic bytes per element)
                    rb = r.element_size() * (9 * s.Np * 2 + 9 * 4 * s.Nfp + 25) + 16
                    rms = timed(lambda: s.elastic_rhs(r, o, wall="free", weighted=False))
                    e[dtype]["rhs_ms"] = rms
                    e[dtype]["rhs_GBps"] = rb * s.K / (rms * 1e-3) / 1e9
                    e[dtype]["rhs_weighted_ms"] = timed(lambda: s.elastic_rhs(r, o, wall="free", weighted=True))
                    res = torch.zeros_like(r)
                    e[dtype]["step_ms"] = timed(lambda: s.elastic_step(r, res, 1e-9, 1, wall="free"))
                    if dtype == "f64":
                        s.project_c2(c2_gaussian_bumps(0))
                        s.dense_set_c2(None)
                        p0 = r[0].contiguous()
                        p1 = torch.empty_like(p0)
                        e["dense_9_updates_ms"] = 9 * timed(lambda: s.dense_update(p0, p1))
                    del s, r, o
                out.append(e)
                print(json.dumps({"elastic_progress": e}), file=sys.stderr, flush=True)
                torch.cuda.empty_cache()
    return out


def c2_bumps_medium():
    from workloads import c2_gaussian_bumps
    return c2_gaussian_bumps(0)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-c1", action="store_true", help="skip the small 384-tet configuration")
    ap.add_argument("--fp32-only", action="store_true", help="time only the FP32 leg (profiling)")
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter reference)")
    ap.add_argument("--cpu-steps", type=int, default=15, help="LSRK4 steps of the CPU oracle sample")
    ap.add_argument("--wadg-compare", action="store_true",
                    help="instead of the default workload: dense quadrature WADG vs the Bernstein update, N = 2..9")
    ap.add_argument("--c3", action="store_true",
                    help="instead of the default workload: N = 4..9, M = N/2 on the three-layer medium, FP64 and FP32")
    ap.add_argument("--c3-n", type=str, default="4,5,6,7,8,9", help="degrees of the --c3 sweep (profiling)")
    ap.add_argument("--wadg-compare-dtypes", type=str, default="f64,f32")
    ap.add_argument("--rates", action="store_true",
                    help="instead of the default workload: manufactured-solution errors and rates, N = 1..6, M = 0..3")
    ap.add_argument("--adjoint", action="store_true",
                    help="instead of the default workload: misfit gradient on 82,944 tets, N=4, M=2, 500 steps")
    ap.add_argument("--adjoint-steps", type=int, default=500)
    ap.add_argument("--wadg-compare-cells", type=int, default=32, help="cube cells per side for --wadg-compare")
    ap.add_argument("--surrogate", action="store_true",
                    help="instead of the default workload: train and score the trace surrogate (256 media)")
    ap.add_argument("--surrogate-media", type=int, default=256)
    ap.add_argument("--elastic", action="store_true",
                    help="instead of the default workload: elastic weight-adjusted update times, N = 2..9, M = 1, 2")
    ap.add_argument("--elastic-only", type=str, default=None, help="one case CELLS,N,M (profiling)")
    ap.add_argument("--surrogate-train-steps", type=int, default=4000)
    ap.add_argument("--fd", type=int, default=20, help="finite-difference checks of the adjoint gradient")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this path has no multi-GPU mode "
              "(elements would be partitioned with one face-trace exchange per stage).", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.wadg_compare:
        res = wadg_compare(range(2, 10), (1, 2), max(1, args.steps), args.wadg_compare_cells,
                           tuple(args.wadg_compare_dtypes.split(",")))
        k = 6 * args.wadg_compare_cells ** 3
        print(json.dumps({"workload": f"cube {args.wadg_compare_cells}^3x6 = {k} tets, bump medium, c^2_M at the dense points",
                          "unit": "ms per evaluation",
                          "reps": max(1, args.steps), "wadg_compare": res}), flush=True)
        return
    if args.elastic:
        only = tuple(int(v) for v in args.elastic_only.split(",")) if args.elastic_only else None
        res = elastic_bench(max(1, min(args.steps, 50)), only)
        print(json.dumps({"workload": "elastic update, right-hand side and step: cubes 11^3x6 and 32^3x6, N=2..9, M=1,2", "unit": "ms per call",
                          "data": "synthetic", "elastic": res}), flush=True)
        return
    if args.surrogate:
        nm = args.surrogate_media
        res = surrogate_bench(nm, nm - max(1, nm // 8), train_steps=args.surrogate_train_steps)
        print(json.dumps({"workload": "surrogate: cube 16^3x6, N=4, M=2, 64 receivers x 400 steps, 256 media",
                          "data": "synthetic", "surrogate": res}), flush=True)
        return
    if args.adjoint:
        res = adjoint_bench(args.adjoint_steps, 50, args.fd)
        print(json.dumps({"workload": f"adjoint: cube 24^3x6, N=4, M=2, 64 receivers, {args.adjoint_steps} steps",
                          "data": "synthetic", "adjoint": res}), flush=True)
        return
    if args.rates:
        res = rates_sweep(range(1, 7), range(0, 4), (2, 4, 8, 16))
        print(json.dumps({"workload": "manufactured solution on the unit cube, T = 0.5, CFL 0.5", "unit": "L2 error",
                          "dtype": "f64", "rates": res}), flush=True)
        return
    if args.c3:
        res = c3_sweep(args.steps, args.warmup, [int(v) for v in args.c3_n.split(",")])
        print(json.dumps({"metric": "GDOF-updates/s per RK step (FP32 vs FP64) + % HBM peak, at stated L2 error",
                          "unit": "GDOF-updates/s", "workload": "cube196k_N4-9_three_layer", "steps": args.steps,
                          "warmup": args.warmup, "data": "synthetic", "c3": res}), flush=True)
        return

    out = {}
    s64, q0 = setup("f32" if args.fp32_only else "f64")
    dt = s64.suggest_dt(0.5)
    K = s64.K
    dofs = K * dimp(N) * 4
    q64, ms, wall, copy_ms, per_step = run_leg(s64, q0, dt, args.steps, args.warmup, chunks=5)
    kernel_ms = (ms - copy_ms) / (5 * args.steps)
    word = 4 if args.fp32_only else 8
    alg = algorithmic_bytes_per_element(N, M, word) * K
    achieved = alg / (kernel_ms * 1e-3) / 1e9
    traffic = measured_traffic("f32" if args.fp32_only else "f64")
    value = dofs * args.steps / (ms * 1e-3) / 1e9
    out.update({
        "metric": "GDOF-updates/s per RK step (FP32 vs FP64) + % HBM peak, at stated L2 error",
        "value": value,
        "unit": "GDOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "ms_per_step_median_of_5_parts": sorted(per_step)[len(per_step) // 2],
        "ms_per_step_parts": per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.fp32_only else "f64",
        "data": "synthetic",
        "config": {"workload": "cube196k_N5_M2", "elements": K, "N": N, "M": M, "dofs": dofs,
                   "medium": "1 + 8 Gaussian bumps (seed 0), projected to P^2", "ic": "Gaussian pulse",
                   "bc": "p=0 walls", "dt": dt, "cfl": 0.5, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "stage_kernel (fused volume + surface/lift + WADG + LSRK stage)",
                     "kernel_ms": kernel_ms,
                     "alg_bytes_per_launch": alg,
                     "alg_bytes_per_element": algorithmic_bytes_per_element(N, M, word),
                     "alg_bytes_formula": "(16 Np + Mp + 25) s + 16 (four int32 neighbour ids)"},
    })
    if not args.no_fp32 and not args.fp32_only:
        s32, _ = setup("f32")
        q32, ms32, _, _, per32 = run_leg(s32, q0, dt, args.steps, args.warmup, chunks=5)
        # both legs advanced warmup + steps steps from the same start
        import torch
        a = q32.double()
        b = q64
        num = torch.sum((a - b) ** 2, dim=(1, 2))
        den = torch.clamp(torch.sum(b ** 2, dim=(1, 2)), min=1e-300)
        rel = torch.sqrt(num / den).cpu().numpy().tolist()
        l2a = s64.l2norm2((a - b).contiguous())
        l2b = s64.l2norm2(b)
        rel_fn = np.sqrt(l2a / np.maximum(l2b, 1e-300)).tolist()
        out["fp32"] = {"value": dofs * args.steps / (ms32 * 1e-3) / 1e9, "ms_per_step": ms32 / args.steps,
                       "ms_per_step_median_of_5_parts": sorted(per32)[len(per32) // 2],
                       "speedup_vs_fp64": ms / ms32,
                       "rel_l2_vs_fp64_per_field": rel_fn,
                       "rel_coef_l2_vs_fp64_per_field": rel,
                       "alg_frac_hbm": algorithmic_bytes_per_element(N, M, 4) * K /
                       ((ms32 / (5 * args.steps)) * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "traffic": measured_traffic("f32")}
    cp = copy_bandwidth()
    out["roofline"]["copy_gbs"] = cp["gbs"]
    out["roofline"]["frac_of_copy"] = achieved / cp["gbs"]
    out["copy_ref"] = cp
    out["l2_error"] = {"fp32_vs_fp64": out.get("fp32", {}).get("rel_l2_vs_fp64_per_field")}
    if not args.no_cpu_baseline:
        xyz, etov = s64._xyz, s64._etov
        out["cpu_baseline"] = cpu_baseline(dt, args.cpu_steps)
        par = {"f64": oracle_parity(s64, xyz, etov, q64)}
        if "fp32" in out:
            par["f32"] = oracle_parity(s32, xyz, etov, q32)
        out["l2_error"]["vs_oracle_sampled"] = par
    if not args.no_c1:
        out["c1"] = c1_entry()
    if args.copy_ref_mib > 0:
        import torch
        n = args.copy_ref_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_ref_counters"] = {"bytes_read": n * 8, "bytes_written": n * 8}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
