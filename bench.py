"""Throughput benchmark of the implicit filter on one MI355X.

Workload: icosahedral sphere, level 9 (2,621,442 vertices), 10% jitter,
40% of the vertices land-masked as 40 seeded caps; 64 scalar fields
(32 depth levels x 2 variables, k^-3 spectra scaled by exp(-z / 1000 m),
z log-spaced 5 m .. 5 km) filtered at 30 wavenumbers (wavelengths
log-spaced 32h .. 2h), order n = 1: 1,920 solves per step. Inputs are
synthetic (seeded) and resident in HBM before the timed region.

Prints one JSON line: solves/s of the whole job (the timed steps), the
roofline of the dominant kernel (algorithmic bytes per launch / mean launch
time from HIP events recorded live on the launch stream; HBM traffic from
the committed rocprofv3 profile; the library's own 4 GiB device copy probe
timed in the same run), and, outside the timed steps: the plain FP64
one-column-at-a-time path on a subset of the fields, SpMV rates on the
unmasked level-9 mesh (single column FP64 / FP32, n = 1, 2 and 4; 32
batched columns), C1 (64 x 64 planar, plain FP64, latency-bound) and C2
(level-8 sphere, n = 2, mixed batched vs plain FP64), velocity filtering on
the level-8 sphere (the vertex FE vector Laplacian fed by the cell -> vertex
projection, and the cell-vector operator of Eq. 7), the continuous-batching
server on resident level 6-10 meshes (200 warm-up + 2,000 measured requests
at 200 req/s, a stream below capacity, a like-for-like comparison with the
plain FP64 path, and the SpMV rates on the level-10 mesh), and the FP64 CPU
oracle on a bounded sample of the same workload (one thread, and one
process per core) together with the GPU's error on it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# rocprofv3 summaries of the default workload (profiles/*.txt): per-launch
# HBM bytes of the batched SpMV kernel from FETCH_SIZE / WRITE_SIZE counters,
# scaled by the counters of a plain device copy of known size
PROFILE_DIR = os.path.join(ROOT, "profiles")


def recorded_traffic(kernel: str):
    """HBM bytes per launch of `kernel` as counted in a committed profile,
    or None if there is none or the kernel source changed since."""
    import glob
    import hashlib

    src = os.path.join(ROOT, "paper_2404_07398_amd", "csrc", "batch.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for path in sorted(glob.glob(os.path.join(PROFILE_DIR, "*.txt"))):
        try:
            kv = {}
            for line in open(path):
                if ":" in line:
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
            if kv.get("kernel_source_sha256") == sha and kv.get("traffic_kernel") == kernel:
                return float(kv["traffic_bytes_per_launch"])
        except (OSError, KeyError, ValueError):
            continue
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(level: int, mask: float, n_fields: int, n_scales: int, device: str):
    import workloads as W

    t0 = time.time()
    s = W.icosphere(level, jitter=0.1, seed=1)
    s = s.with_mask(W.land_mask(s, mask, n_blobs=40, seed=2))
    ks = W.log_scales(s.h, n_scales)
    depths = 5.0 * 1000.0 ** (np.arange(32) / 31.0)
    fields = []
    for f in range(n_fields):
        lvl, var = f // 2, f % 2
        phi = W.sphere_k3_field(s, 1000 + f, n_waves=512, device=device)
        fields.append(phi * math.exp(-depths[lvl % 32] / 1000.0))
    log(f"workload generated in {time.time() - t0:.1f}s: V={s.n_vertices} F={s.n_triangles}")
    return s, np.stack(fields), ks


def cpu_baseline(mesh, fields, ks, budget_s: float = 20.0, gpu_column=None):
    """The FP64 oracle on a bounded sample: solves of field 0 at scales
    taken alternately from both ends of the k list, until the budget is
    spent (at least one solve). With gpu_column(j) (the GPU's result for
    field 0 at scale j, caller numbering), also the relative L2 error of the
    GPU results on that sample (not timed)."""
    import oracle as O
    from oracle.solve import relative_l2

    t0 = time.time()
    op = O.scalar_operator(mesh, 1)
    t_prep = time.time() - t0
    order = []
    lo, hi = 0, len(ks) - 1
    while lo <= hi:
        order.append(lo)
        if hi != lo:
            order.append(hi)
        lo, hi = lo + 1, hi - 1
    done = 0
    t1 = time.time()
    sols = []
    for j in order:
        sols.append((j, O.filter_scalar(op, fields[0], [ks[j]])[0]))
        done += 1
        if time.time() - t1 > budget_s:
            break
    el = time.time() - t1
    parity = None
    if gpu_column is not None:
        errs = [relative_l2(gpu_column(j), x) for j, x in sols]
        parity = {"max_rel_l2": float(max(errs)), "solves": len(errs), "tol": 1e-9,
                  "what": "GPU result of the benchmark's launch configuration vs the FP64 oracle on the "
                          "baseline's sample (field 0)"}
    return parity, {
        "value": done / el,
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{done} solves of field 0 (scales alternating from both ends of the k list) on the "
                  f"same level-9 masked mesh, NumPy/SciPy FP64 Jacobi-PCG + extended-precision refinement, "
                  f"single-threaded sparse products; oracle prepare {t_prep:.1f}s not counted",
    }


def spmv_leg(ifl):
    """SpMV rates on the unmasked level-9 icosphere (2,621,442 vertices, all
    of them dofs): the single-column kernels in FP64 and FP32 for n = 1, 2
    and 4 (K_4: up to 61 entries a row), and the batched kernel (32 mixed
    columns) for n = 1. Each figure is algorithmic bytes per launch over the
    HIP-event time of the launch."""
    import torch

    import workloads as W

    s = W.icosphere(9, jitter=0.1, seed=1)
    phi = torch.from_numpy(np.asarray(W.sphere_k3_field(s, 1000, n_waves=512, device="cuda:0"))).to("cuda:0")
    lam = [32, 16, 8, 4]
    ks = np.array([2 * math.pi / (x * s.h) for x in lam])
    res = {"vertices": s.n_vertices, "scales": f"wavelengths {lam} h"}

    def timed(h, fields, kk):
        nf = fields.shape[0] if fields.dim() == 2 else 1
        dst = torch.empty((nf, len(kk), h.field_length), dtype=torch.float64, device="cuda:0")
        h.filter(fields, kk[:1], out=torch.empty((nf, 1, h.field_length), dtype=torch.float64, device="cuda:0"))
        h.profile_read(reset=True)
        _, st = h.filter(fields, kk, out=dst)
        n, ms, b = h.profile_read(reset=True)
        us = ms / max(n, 1) * 1e3
        return {"kernel": h.profile_kernel(), "mean_launch_us": round(us, 2), "bytes_per_launch": round(b),
                "GBs": round(b / (us * 1e3), 1) if n else None,
                "frac_of_hbm_peak": round(b / (us * 1e3) / HBM_PEAK_GBS, 4) if n else None, "launches": n,
                "mean_cg_iterations": round(sum(x.iterations for x in st) / len(st), 1)}

    for n in (1, 2, 4):
        t0 = time.time()
        h = ifl.prepare_mesh(s, ifl.IFL_VERTEX_SCALAR, n, precision=ifl.IFL_FP64, batch=1, device=0, profile=1)
        res[f"n{n}_prepare_s"] = round(time.time() - t0, 1)
        kk = ks if n == 1 else ks[2:]  # n = 2, 4: the smaller scales keep the iteration count modest
        for prec, name in ((ifl.IFL_FP64, "fp64"), (ifl.IFL_MIXED, "fp32")):
            h.set_options(precision=prec, batch=1)
            res[f"n{n}_{name}_single_column"] = timed(h, phi, kk)
        if n == 1:
            # 32 copies of the field at one scale: every timed launch has all 32 columns live
            h.set_options(precision=ifl.IFL_MIXED, batch=32)
            many = phi.unsqueeze(0).expand(32, -1).contiguous()
            res["n1_fp32_batched_32"] = timed(h, many, ks[1:2].repeat(2))
        h.close()
    return res


def spmv10_leg(ifl):
    """Out-of-cache cross-check of the single-column iteration rates: the
    unmasked level-10 icosphere (10,485,762 vertices, all dofs), n = 1, FP64
    and FP32, two scales (wavelengths 16h, 8h). Algorithmic bytes per
    launch (1.5 GB FP64) are ~6x the 256 MB Infinity Cache, so the rate is
    an HBM rate."""
    import torch

    import workloads as W

    s = W.icosphere(10, jitter=0.1, seed=1)
    phi = torch.from_numpy(np.asarray(W.sphere_k3_field(s, 1000, n_waves=256, device="cuda:0"))).to("cuda:0")
    ks = np.array([2 * math.pi / (16 * s.h), 2 * math.pi / (8 * s.h)])
    t0 = time.time()
    h = ifl.prepare_mesh(s, ifl.IFL_VERTEX_SCALAR, 1, precision=ifl.IFL_FP64, batch=1, device=0, profile=1)
    res = {"vertices": s.n_vertices, "dofs": h.num_dofs, "prepare_s": round(time.time() - t0, 1),
           "scales": "wavelengths [16, 8] h"}
    dst = torch.empty((1, 2, h.field_length), dtype=torch.float64, device="cuda:0")
    for prec, name in ((ifl.IFL_FP64, "fp64_single_column"), (ifl.IFL_MIXED, "fp32_single_column")):
        h.set_options(precision=prec, batch=1, profile=1)
        h.filter(phi, ks[:1], out=dst[:, :1])
        h.profile_read(reset=True)
        _, st = h.filter(phi, ks, out=dst)
        n_l, ms, b = h.profile_read(reset=True)
        us = ms / max(n_l, 1) * 1e3
        res[name] = {"kernel": h.profile_kernel(), "mean_launch_us": round(us, 2), "bytes_per_launch": round(b),
                     "GBs": round(b / (us * 1e3), 1) if n_l else None,
                     "frac_of_hbm_peak": round(b / (us * 1e3) / HBM_PEAK_GBS, 4) if n_l else None,
                     "launches": n_l, "mean_cg_iterations": round(sum(x.iterations for x in st) / len(st), 1)}
    h.close()
    return res


def reach_leg(ifl):
    """Reach of orders 2-4 at large scales: the uniform periodic 64 x 64
    split square (h = 1), one k^-3 field, wavelengths 8h, 11.3h, 16h, 22.6h
    and 32h, Jacobi-PCG on K_n against the shifted first-order solves, FP64
    and mixed, single column, max_iter 20,000. The error is against the
    exact filter on that lattice: each Fourier mode times
    1 / (1 + gamma (lam / k^2)^n), lam = 4 sin^2(qx/2) + 4 sin^2(qy/2)."""
    import workloads as W

    N = 64
    m = W.split_square(N, jitter=0.0)
    phi = W.planar_k3_field(m, 1000)
    lams = [8.0, 8.0 * math.sqrt(2.0), 16.0, 16.0 * math.sqrt(2.0), 32.0]
    ks = np.array([2 * math.pi / wl for wl in lams])
    q = 2 * np.pi * np.fft.fftfreq(N)
    QX, QY = np.meshgrid(q, q)
    lam = 4 * np.sin(QX / 2) ** 2 + 4 * np.sin(QY / 2) ** 2
    F = np.fft.fft2(phi.reshape(N, N))
    res = {"mesh": "uniform periodic 64 x 64 split square", "wavelengths_h": [round(x, 1) for x in lams]}
    for n in (2, 3, 4):
        for solver, sname in ((ifl.IFL_SOLVER_KN, "kn"), (ifl.IFL_SOLVER_SHIFTED, "shifted")):
            for prec, pname in ((ifl.IFL_FP64, "fp64"), (ifl.IFL_MIXED, "mixed")):
                h = ifl.prepare_mesh(m, ifl.IFL_VERTEX_SCALAR, n, precision=prec, batch=1, device=0,
                                     solver=solver, max_iter=20000)
                t = time.perf_counter()
                out, st = h.filter(phi, ks, raise_on_notconv=False)
                el = time.perf_counter() - t
                h.close()
                errs = []
                for j, k in enumerate(ks):
                    ref = np.real(np.fft.ifft2(F / (1.0 + 0.5 * (lam / k ** 2) ** n))).ravel()
                    errs.append(float("%.1e" % (np.linalg.norm(out[0, j] - ref) / np.linalg.norm(ref))))
                res[f"n{n}_{sname}_{pname}"] = {
                    "status": [int(x.status) for x in st], "iterations": [int(x.iterations) for x in st],
                    "rel_err": errs, "solves_per_s": round(len(ks) / el, 1)}
    return res


def vector_leg(ifl):
    """Velocity filtering on the level-8 sphere (655,362 vertices,
    1,310,720 triangles; 30% land and dry polar caps, where lon/lat
    components are singular): 8 k^-3 velocity fields (rotational + 10%
    divergent) x 8 scales (wavelengths 32h .. 2h), n = 1, mixed precision,
    auto-width tiles, one ifl_filter call. Vertex vectors (Sect. 2.1.2) take
    the cell velocities through ifl_project_cells (timed on its own); cell
    vectors (Eq. 7) filter them in place. Fields are resident in HBM."""
    import torch

    import workloads as W

    s = W.icosphere(8, jitter=0.1, seed=1)
    wet = np.array(W.land_mask(s, 0.3, n_blobs=40, seed=2), dtype=np.uint8)
    wet[np.abs(s.coords[:, 2] / s.radius) > math.sin(math.radians(80))] = 0
    s = s.with_mask(wet)
    nf = 8
    cells = torch.stack([torch.from_numpy(np.asarray(W.sphere_k3_velocity(s, 100 + i, 200 + i, n_waves=256,
                                                                          device="cuda:0")).reshape(-1))
                         for i in range(nf)]).to("cuda:0")
    ks = W.log_scales(s.h, 8)
    res = {"vertices": s.n_vertices, "triangles": s.n_triangles, "fields": nf, "scales": int(ks.size)}
    for placement, name in ((ifl.IFL_VERTEX_VECTOR, "vertex_vector"), (ifl.IFL_CELL_VECTOR, "cell_vector")):
        t0 = time.time()
        h = ifl.prepare_mesh(s, placement, 1, precision=ifl.IFL_MIXED, device=0)
        prep = time.time() - t0
        h.set_options(profile=0)
        L = h.field_length
        fields = torch.empty((nf, L), dtype=torch.float64, device="cuda:0")
        proj_ms = None
        if placement == ifl.IFL_VERTEX_VECTOR:
            h.project_cells(cells[0], out=fields[0])
            torch.cuda.synchronize()
            t = time.perf_counter()
            for i in range(nf):
                h.project_cells(cells[i], out=fields[i])
            torch.cuda.synchronize()
            proj_ms = (time.perf_counter() - t) / nf * 1e3
        else:
            fields.copy_(cells)
        dst = torch.empty((nf, ks.size, L), dtype=torch.float64, device="cuda:0")
        h.filter(fields, ks, out=dst)  # untimed: the same call, so the tile of its width exists
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st = h.filter(fields, ks, out=dst)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        res[name] = {"solves_per_s": round(nf * ks.size / el, 2), "unknowns": h.num_dofs,
                     "mean_cg_iterations": round(sum(x.iterations for x in st) / len(st), 1),
                     "prepare_s": round(prep, 1)}
        # the same call again with HIP events around the tile's SpMV launches
        # (not timed above): algorithmic bytes per launch / mean launch time
        h.set_options(profile=1)
        h.profile_read(reset=True)
        h.filter(fields, ks, out=dst)
        nl, ms, b = h.profile_read(reset=True)
        h.set_options(profile=0)
        if nl:
            us = ms / nl * 1e3
            gbs = b / (us * 1e3)
            res[name]["roofline"] = {"bound": "hbm", "kernel": h.profile_kernel(), "launches": nl,
                                     "mean_launch_us": round(us, 2), "bytes_per_launch": round(b),
                                     "achieved_GBs": round(gbs, 1), "peak_GBs": HBM_PEAK_GBS,
                                     "frac": round(gbs / HBM_PEAK_GBS, 4)}
        if proj_ms is not None:
            res[name]["project_cells_ms"] = round(proj_ms, 3)
        h.close()
        del fields, dst
    return res


def c1_leg(ifl):
    """C1, the latency-bound configuration: 64 x 64 periodic split-square
    mesh (4,096 vertices, jitter +-0.2 cell), one k^-3 field, n = 1, 8
    scales (wavelengths 32 .. 2 cells), the plain FP64 path one column at a
    time. One SpMV moves ~0.5 MB, so the rate is set by launch and reduction
    latency, not bandwidth. Field and outputs resident on the device."""
    import torch

    import workloads as W

    m = W.split_square(64, jitter=0.2, seed=1)
    phi = torch.from_numpy(W.planar_k3_field(m, 1000)).to("cuda:0")
    ks = W.log_scales(1.0, 8)
    res = {"workload": "64x64 periodic split square (4,096 vertices, jitter 0.2), 1 k^-3 field x 8 scales "
                       "(wavelengths 32..2 cells), n=1"}
    for prec, batch, name in ((ifl.IFL_FP64, 1, "fp64_single_column"), (ifl.IFL_MIXED, 0, "mixed_batched")):
        h = ifl.prepare_mesh(m, ifl.IFL_VERTEX_SCALAR, 1, precision=prec, batch=batch, device=0)
        out = torch.empty((1, ks.size, h.field_length), dtype=torch.float64, device="cuda:0")
        h.filter(phi, ks, out=out)
        torch.cuda.synchronize()
        reps = 20
        t = time.perf_counter()
        iters = 0
        for _ in range(reps):
            _, st = h.filter(phi, ks, out=out)
            iters += sum(x.iterations for x in st)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        res[name] = {"solves_per_s": round(reps * ks.size / el, 1),
                     "ms_per_solve": round(el / (reps * ks.size) * 1e3, 3),
                     "mean_cg_iterations": round(iters / (reps * ks.size), 1),
                     "us_per_iteration": round(el / max(1, iters) * 1e6, 2)}
        h.close()
    return res


def c2_leg(ifl):
    """C2: level-8 icosphere (655,362 vertices), 10% jitter, 30% land mask
    (40 caps), one k^-3 field, n = 2 (biharmonic), 20 scales (wavelengths
    32h .. 2h): the batched mixed-precision form (auto tile width) against
    the plain FP64 path one column at a time, same GPU, same call; and the
    same solves as one complex-shifted first-order system each
    (IFL_SOLVER_SHIFTED, FP64 and mixed). The
    matrix of K_2 (~8.5 M entries) and the vectors largely fit the 256 MB
    Infinity Cache, so rates are not HBM rates."""
    import torch

    import workloads as W

    s = W.icosphere(8, jitter=0.1, seed=1)
    s = s.with_mask(W.land_mask(s, 0.3, n_blobs=40, seed=2))
    phi = torch.from_numpy(np.asarray(W.sphere_k3_field(s, 1000, n_waves=512, device="cuda:0"))).to("cuda:0")
    ks = W.log_scales(s.h, 20)
    h = ifl.prepare_mesh(s, ifl.IFL_VERTEX_SCALAR, 2, precision=ifl.IFL_MIXED, device=0)
    res = {"workload": f"icosphere-L8 {s.n_vertices} vertices, 30% land mask ({h.num_dofs} dofs), n=2, "
                       f"1 k^-3 field x 20 scales (wavelengths 32h..2h)"}
    out = torch.empty((1, ks.size, h.field_length), dtype=torch.float64, device="cuda:0")
    for prec, batch, solver, name in ((ifl.IFL_MIXED, 0, 0, "mixed_batched"), (ifl.IFL_FP64, 1, 0, "fp64_single_column"),
                                      (ifl.IFL_FP64, 1, 1, "shifted_fp64_single_column"),
                                      (ifl.IFL_MIXED, 1, 1, "shifted_mixed_single_column"),
                                      (ifl.IFL_FP64, 0, 1, "shifted_fp64_complex_tiles"),
                                      (ifl.IFL_MIXED, 0, 1, "shifted_mixed_complex_tiles")):
        h.set_options(precision=prec, batch=batch, solver=solver)
        h.filter(phi, ks, out=out)  # untimed: the same call, so the tile of its width exists
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st = h.filter(phi, ks, out=out)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        res[name] = {"solves_per_s": round(ks.size / el, 2),
                     "mean_cg_iterations": round(sum(x.iterations for x in st) / len(st), 1),
                     "max_cg_iterations": int(max(x.iterations for x in st)),
                     "fp64_replacements": int(sum(x.refinements for x in st))}
    res["speedup_mixed_batched_vs_plain_fp64"] = round(res["mixed_batched"]["solves_per_s"] /
                                                       res["fp64_single_column"]["solves_per_s"], 3)
    res["speedup_shifted_fp64_vs_plain_fp64"] = round(res["shifted_fp64_single_column"]["solves_per_s"] /
                                                      res["fp64_single_column"]["solves_per_s"], 3)
    res["speedup_shifted_mixed_tiles_vs_plain_fp64"] = round(res["shifted_mixed_complex_tiles"]["solves_per_s"] /
                                                            res["fp64_single_column"]["solves_per_s"], 3)
    res["shifted"] = ("IFL_SOLVER_SHIFTED: S^-1 = Re (M + i c^(1/2) K)^-1 for n = 2, one complex-shifted "
                      "first-order system per solve, Jacobi-COCG, one column at a time (batch 1) or in complex "
                      "tiles (auto width)")
    h.close()
    return res


def serve_leg(args, ifl):
    """Continuous-batching server (C5): resident prepared meshes (icosphere
    levels 6..10, 30% land, each prepared for n = 1 and n = 2, mixed
    precision, 8 column slots per mesh), a memory budget for admission, and
    Poisson arrival streams. Each request: a uniform mesh handle, 1-32
    log-uniform scales in [2h, 32h] wavelengths, a field from a pool of 4 per
    mesh. Streams: (1) the stated one, 200 warm-up + 2,000 measured requests
    at 200 req/s, spectrum-only (the energies of the filtered fields, so that
    an overloaded queue does not hold up to 32 x 84 MB of outputs per
    level-10 request), in a bounded window: what has not finished 20 s after
    the last arrival is cancelled and reported as such; (2) a stream below
    capacity with the filtered fields returned. Then a like-for-like comparison on one request sample (served,
    fields returned, vs the plain FP64 path one column at a time), and the
    out-of-cache SpMV rates on the level-10 mesh."""
    import threading

    import torch

    import workloads as W

    levels = [int(x) for x in args.serve_levels.split(",") if x]
    rng = np.random.default_rng(7)
    handles, meshes, pools = [], [], []
    t0 = time.time()
    for L in levels:
        s = W.icosphere(L, jitter=0.1, seed=1)
        s = s.with_mask(W.land_mask(s, 0.3, n_blobs=40, seed=2))
        pool = [np.asarray(W.sphere_k3_field(s, 3000 + 10 * L + i, n_waves=256, device="cuda:0"))
                for i in range(4)]
        for n in (1, 2):
            solver = ifl.IFL_SOLVER_SHIFTED if (n == 2 and args.serve_n2_solver == "shifted") else ifl.IFL_SOLVER_KN
            handles.append(ifl.prepare_mesh(s, ifl.IFL_VERTEX_SCALAR, n, precision=ifl.IFL_MIXED, device=0,
                                            graphs=0 if args.no_graphs else 1, solver=solver))
            meshes.append((L, n, s.h))
            pools.append(pool)
        log(f"serving: level {L} prepared ({time.time() - t0:.1f}s)")
    prep_s = time.time() - t0
    srv = ifl.Server(int(args.serve_budget_gib * (1 << 30)), slots=args.serve_slots)
    ids = [srv.add(h) for h in handles]
    for i, (L, n, h) in enumerate(meshes):  # warm every worker once
        t, _ = srv.submit(ids[i], pools[i][0], np.array([2 * math.pi / (4 * h)]))
        srv.wait(t, 1)

    def draw(N):
        reqs = []
        for _ in range(N):
            i = int(rng.integers(len(handles)))
            L, n, h = meshes[i]
            ns = int(rng.integers(1, 33))
            ks = np.sort(np.exp(rng.uniform(math.log(2 * math.pi / (32 * h)), math.log(2 * math.pi / (2 * h)), ns)))
            reqs.append((i, int(rng.integers(4)), ks))
        return reqs

    def stream(rate, reqs, warmup, spectrum_only, drain_s=None):
        # a waiter thread takes the tickets in submission order while the
        # arrivals go on, so finished outputs are dropped at once
        arrivals = np.cumsum(rng.exponential(1.0 / rate, len(reqs)))
        box = []
        cv = threading.Condition()
        done = {}

        def waiter():
            k = 0
            t_log = time.perf_counter()
            while k < len(reqs):
                with cv:
                    while len(box) <= k:
                        cv.wait()
                    t, ns, i, t_sub = box[k]
                st, stats, out, lat = srv.wait(t, ns)
                done[k] = (st, ns, i, lat, sum(x.iterations for x in stats), t_sub + lat)
                del out
                k += 1
                if time.perf_counter() - t_log > 10.0:
                    t_log = time.perf_counter()
                    log(f"  stream at {rate:g}/s: {k}/{len(reqs)} requests done, {len(box)} submitted")

        th = threading.Thread(target=waiter, daemon=True)
        th.start()
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        lag = 0.0
        for r, (i, f, ks) in enumerate(reqs):
            delay = arrivals[r] - (time.perf_counter() - t_start)
            if delay > 0:
                time.sleep(delay)
            else:
                lag = max(lag, -delay)
            t_sub = time.perf_counter() - t_start
            t, _ = srv.submit(ids[i], pools[i][f], ks, spectrum_only=spectrum_only)
            with cv:
                box.append((t, ks.size, i, t_sub))
                cv.notify()
        cancelled_at = None
        if drain_s is not None:
            # bounded window: what has not finished drain_s after the last
            # arrival is cancelled (its latency is only known to exceed the
            # window)
            th.join(timeout=max(0.0, float(arrivals[-1]) + drain_s - (time.perf_counter() - t_start)))
            if th.is_alive():
                cancelled_at = time.perf_counter() - t_start
                log(f"  stream at {rate:g}/s: window over, cancelling what has not started")
                srv.cancel()
        # columns already running finish after a cancel; a stream that still
        # has not drained after this long is reported as stuck
        th.join(timeout=max(120.0, 2.0 * float(arrivals[-1])) if drain_s is not None else None)
        if th.is_alive():
            raise RuntimeError(f"serving stream at {rate:g}/s did not drain: {len(done)}/{len(reqs)} requests "
                               f"finished 120 s after the cancel")
        meas = [done[k] for k in range(warmup, len(reqs))]
        ok = [x for x in meas if x[0] == 0]
        t_first = float(arrivals[warmup])
        t_last = max(x[5] for x in ok) if ok else t_first
        span = max(1e-9, (cancelled_at if cancelled_at is not None else t_last) - t_first)
        # latencies of cancelled requests are censored (> their time in the window)
        lat = np.sort(np.array([x[3] if x[0] == 0 else np.inf for x in meas]))

        def pct(p):
            v = float(lat[min(len(lat) - 1, int(math.ceil(p / 100.0 * len(lat))) - 1)])
            return round(v * 1e3, 2) if math.isfinite(v) else None

        per = {}
        for x in ok:
            per.setdefault(meshes[x[2]][:2], []).append(x[3])
        solves = sum(x[1] for x in ok)
        # completion rate while requests still arrive (the service rate once
        # the queue has built up)
        t_arr_end = float(arrivals[-1])
        in_window = sum(1 for x in ok if x[5] <= t_arr_end)
        return {
            "drain_lag_s": round(t_last - t_arr_end, 3) if ok else None,
            "in_window_rate_req_s": round(in_window / max(1e-9, t_arr_end - t_first), 2),
            "p50_latency_ms": pct(50),
            "p99_latency_ms": pct(99),
            "solves_per_s": round(solves / span, 2),
            "requests": len(meas),
            "completed_requests": len(ok),
            "cancelled_requests": int(sum(x[0] == ifl.IFL_ECANCELED for x in meas)),
            "window_s": round(cancelled_at - t_first, 3) if cancelled_at is not None else None,
            "warmup_requests": warmup,
            "failed": int(sum(x[0] not in (0, ifl.IFL_ECANCELED) for x in meas)),
            "offered_rate_req_s": rate,
            "achieved_rate_req_s": round(len(ok) / span, 2),
            "arrival_window_s": round(float(arrivals[-1] - arrivals[warmup]), 3),
            "measured_span_s": round(span, 3),
            "max_submit_lag_s": round(lag, 4),
            "solves": int(solves),
            "mean_cg_iterations": round(sum(x[4] for x in meas) / max(1, solves), 1),
            "p50_latency_ms_by_mesh": {f"L{L}-n{n}": round(float(np.percentile(v, 50)) * 1e3, 1)
                                       for (L, n), v in sorted(per.items())},
            "outputs": "spectrum only (energies)" if spectrum_only else "filtered fields to host",
        }

    res = {"workload": f"icosphere levels {args.serve_levels} (30% land mask) x n in {{1,2}}, "
                       f"{args.serve_slots} slots per mesh, mixed precision, 1-32 log-uniform scales per request; "
                       + ("n = 2 requests by the shifted first-order solves in complex tiles"
                          if args.serve_n2_solver == "shifted" else "n = 2 requests by Jacobi-PCG on K_2 in tiles"),
           "prepare_s": round(prep_s, 1), "budget_bytes": int(args.serve_budget_gib * (1 << 30))}
    res["stream"] = stream(args.serve_rate, draw(args.serve_warmup + args.serve_requests), args.serve_warmup, True,
                           drain_s=args.serve_drain_s)
    q = srv.query()
    res["memory"] = {"tiles_bytes": q["tiles"], "peak_request_bytes": q["peak_used"],
                     "peak_in_flight": q["peak_in_flight"]}
    log(f"serving at {args.serve_rate:g}/s: {res['stream']}")
    if args.serve_sustained_rate > 0 and args.serve_sustained_requests > 0:
        res["sustained"] = stream(args.serve_sustained_rate, draw(args.serve_sustained_requests), 0, False)
        log(f"serving at {args.serve_sustained_rate:g}/s: {res['sustained']}")
    if args.serve_sweep:
        # rising offered rates (spectrum-only, bounded window); a rate is
        # sustained when nothing is cancelled or failed and requests complete
        # at >= 0.85 x the offered rate while they arrive (a server that
        # falls behind completes at its service rate, and its queue grows);
        # the sweep stops at the first rate that is not
        pts = []
        for rate in [float(x) for x in args.serve_sweep.split(",") if x]:
            r = stream(rate, draw(args.serve_sweep_requests), 0, True, drain_s=args.serve_sweep_drain_s)
            ok = (r["cancelled_requests"] == 0 and r["failed"] == 0
                  and r["in_window_rate_req_s"] >= 0.85 * rate)
            pts.append({"offered_rate_req_s": rate, "in_window_rate_req_s": r["in_window_rate_req_s"],
                        "achieved_rate_req_s": r["achieved_rate_req_s"], "drain_lag_s": r["drain_lag_s"],
                        "p50_latency_ms": r["p50_latency_ms"], "p99_latency_ms": r["p99_latency_ms"],
                        "completed_requests": r["completed_requests"], "requests": r["requests"],
                        "solves_per_s": r["solves_per_s"], "sustained": ok})
            log(f"serving sweep: {pts[-1]}")
            if not ok:
                break
        res["rate_sweep"] = {
            "requests_per_rate": args.serve_sweep_requests, "drain_s": args.serve_sweep_drain_s,
            "rule": "sustained: no request cancelled or failed, and requests completed at >= 0.85 x the offered "
                    "rate while they arrived",
            "points": pts,
            "highest_sustained_rate_req_s": max([x["offered_rate_req_s"] for x in pts if x["sustained"]],
                                                default=None)}
    # like-for-like: one request sample, served (fields returned) and plain FP64
    cmp_reqs = draw(args.serve_compare) if args.serve_compare > 0 else []
    if cmp_reqs:
        t = time.perf_counter()
        tl = [srv.submit(ids[i], pools[i][f], ks) for (i, f, ks) in cmp_reqs]
        for (tk, _), (_, _, ks) in zip(tl, cmp_reqs):
            srv.wait(tk, ks.size)
        served_s = time.perf_counter() - t
    srv.close()
    if cmp_reqs:
        solves = sum(ks.size for (_, _, ks) in cmp_reqs)
        t = time.perf_counter()
        for r, (i, f, ks) in enumerate(cmp_reqs):
            h = handles[i]
            h.set_options(precision=ifl.IFL_FP64, batch=1, solver=ifl.IFL_SOLVER_KN)
            h.filter(pools[i][f], ks)
            log(f"like-for-like: plain FP64 request {r + 1}/{len(cmp_reqs)} (L{meshes[i][0]} n={meshes[i][1]}, "
                f"{ks.size} scales) done at {time.perf_counter() - t:.1f}s")
        plain_s = time.perf_counter() - t
        for h, (L, n, _) in zip(handles, meshes):
            h.set_options(precision=ifl.IFL_MIXED, batch=0,
                          solver=ifl.IFL_SOLVER_SHIFTED if (n == 2 and args.serve_n2_solver == "shifted")
                          else ifl.IFL_SOLVER_KN)
        res["like_for_like"] = {"requests": len(cmp_reqs), "solves": int(solves),
                                "served_mixed_solves_per_s": round(solves / served_s, 2),
                                "plain_fp64_single_column_solves_per_s": round(solves / plain_s, 2),
                                "speedup": round(plain_s / served_s, 3),
                                "what": "the same requests (fields to host) served together by the server vs "
                                        "one ifl_filter call per request with the plain FP64 path"}
        log(f"serving like-for-like: {res['like_for_like']}")
    # out-of-cache SpMV rates: the level-10 mesh (n = 1) of the server
    if 10 in levels:
        i10 = meshes.index(next(m for m in meshes if m[0] == 10 and m[1] == 1))
        h = handles[i10]
        L, _, hh = meshes[i10]
        ks = np.array([2 * math.pi / (16 * hh), 2 * math.pi / (8 * hh)])
        f = torch.from_numpy(pools[i10][0]).to("cuda:0")
        dst = torch.empty((1, 2, h.field_length), dtype=torch.float64, device="cuda:0")
        sp = {"dofs": h.num_dofs}
        for prec, name in ((ifl.IFL_FP64, "fp64_single_column"), (ifl.IFL_MIXED, "fp32_single_column")):
            h.set_options(precision=prec, batch=1, profile=1)
            h.filter(f, ks[:1], out=dst[:, :1])
            h.profile_read(reset=True)
            h.filter(f, ks, out=dst)
            n_l, ms, b = h.profile_read(reset=True)
            us = ms / max(n_l, 1) * 1e3
            sp[name] = {"kernel": h.profile_kernel(), "mean_launch_us": round(us, 2), "bytes_per_launch": round(b),
                        "GBs": round(b / (us * 1e3), 1) if n_l else None,
                        "frac_of_hbm_peak": round(b / (us * 1e3) / HBM_PEAK_GBS, 4) if n_l else None,
                        "launches": n_l}
        h.set_options(precision=ifl.IFL_MIXED, batch=0, profile=0, solver=ifl.IFL_SOLVER_KN)
        res["spmv_level10"] = sp
        log(f"level-10 SpMV: {sp}")
    for h in handles:
        h.close()
    return res


def _oracle_worker(task):
    level, mask, field, ks, js, budget = task
    import oracle as O
    import workloads as W

    s = W.icosphere(level, jitter=0.1, seed=1)
    s = s.with_mask(W.land_mask(s, mask, n_blobs=40, seed=2))
    op = O.scalar_operator(s, 1)
    t0 = time.time()
    done = 0
    for j in js:
        O.filter_scalar(op, field, [ks[j]])
        done += 1
        if time.time() - t0 > budget:
            break
    return done, time.time() - t0


def cpu_parallel(level, mask, field, ks, budget_s, workers):
    """The oracle on all host cores: one worker process per core (started
    fresh, single-threaded), each solving its own columns of field 0 for
    about budget_s seconds; aggregate solves/s."""
    import concurrent.futures as cf
    import multiprocessing as mp

    order = []
    lo, hi = 0, len(ks) - 1
    while lo <= hi:
        order.append(lo)
        if hi != lo:
            order.append(hi)
        lo, hi = lo + 1, hi - 1
    tasks = [(level, mask, field, ks, order[w::workers] or order[:1], budget_s) for w in range(workers)]
    env = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env:
        os.environ[k] = "1"
    try:
        with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
            out = list(ex.map(_oracle_worker, tasks))
    finally:
        for k, v in env.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return sum(d / el for d, el in out if el > 0), sum(d for d, _ in out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="mixed")
    ap.add_argument("--batch", type=int, default=0, help="columns per tile (0 = auto)")
    ap.add_argument("--level", type=int, default=9)
    ap.add_argument("--mask", type=float, default=0.4)
    ap.add_argument("--fields", type=int, default=64)
    ap.add_argument("--scales", type=int, default=30)
    ap.add_argument("--field-block", type=int, default=16, help="fields per ifl_filter call")
    ap.add_argument("--plain-fields", type=int, default=4,
                    help="fields for the plain FP64 single-column comparison (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-autotune", action="store_true", help="skip ifl_autotune (default tile and grids)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-spmv-leg", action="store_true", help="skip the SpMV rates on the unmasked level-9 mesh")
    ap.add_argument("--no-vector-leg", action="store_true", help="skip the velocity filtering on the level-8 mesh")
    ap.add_argument("--leg", choices=["velocity", "spmv", "spmv10", "c1", "c2", "reach", "serve"], default=None,
                    help="run only this leg and print its JSON (for profiling one leg on its own)")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch every kernel directly instead of replaying captured chunks")
    ap.add_argument("--serve-levels", default="6,7,8,9,10",
                    help="icosphere levels of the resident meshes (each prepared for n = 1 and n = 2)")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="mean Poisson arrival rate, requests/s")
    ap.add_argument("--serve-requests", type=int, default=2000, help="measured requests in the arrival stream")
    ap.add_argument("--serve-warmup", type=int, default=200, help="requests of the stream before the measured ones")
    ap.add_argument("--serve-slots", type=int, default=8, help="column slots per resident mesh")
    ap.add_argument("--serve-budget-gib", type=float, default=16.0, help="device memory budget of the server")
    ap.add_argument("--serve-sweep", default="4,8,12,16,24,32,48",
                    help="offered rates (req/s) of the serving rate sweep, comma-separated; empty = no sweep")
    ap.add_argument("--serve-sweep-requests", type=int, default=60)
    ap.add_argument("--serve-sweep-drain-s", type=float, default=8.0)
    ap.add_argument("--serve-n2-solver", choices=["shifted", "kn"], default="shifted",
                    help="how the served n = 2 requests are solved: the shifted first-order solves (one column at "
                         "a time) or Jacobi-PCG on K_2 in tiles")
    ap.add_argument("--serve-drain-s", type=float, default=20.0,
                    help="the stated stream's window: requests not finished this long after the last arrival "
                         "are cancelled and counted as such (their latency exceeds the window)")
    ap.add_argument("--serve-sustained-rate", type=float, default=8.0,
                    help="second arrival stream, below the server's capacity, fields returned (req/s; 0 = skip)")
    ap.add_argument("--serve-sustained-requests", type=int, default=100)
    ap.add_argument("--serve-compare", type=int, default=16,
                    help="requests of the served vs plain FP64 comparison (0 = skip)")
    ap.add_argument("--no-c1c2", action="store_true", help="skip the C1 and C2 legs")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="worker processes of the all-cores oracle timing (0 = min(16, host CPUs))")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run the library's plain device copy of this size (a known-traffic kernel "
                         "for calibrating HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the filter's independent "
              "solves would be dealt out per GPU with no communication; the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2404_07398_amd as ifl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    if args.copy_probe_mib > 0:
        # two dispatches of the library's copy kernel (k_stream_copy) of known size
        ifl.stream_probe(0, args.copy_probe_mib, 1)
        log(f"copy probe: 2 x {args.copy_probe_mib} MiB device copies (k_stream_copy)")
    if args.leg is not None:
        fn = {"velocity": vector_leg, "spmv": spmv_leg, "spmv10": spmv10_leg, "c1": c1_leg, "c2": c2_leg,
              "reach": reach_leg,
              "serve": lambda m: serve_leg(args, m)}[args.leg]
        print(json.dumps({"leg": args.leg, **fn(ifl)}), flush=True)
        return
    mesh, fields_h, ks = make_workload(args.level, args.mask, args.fields, args.scales, dev)
    precision = ifl.IFL_MIXED if args.precision == "mixed" else ifl.IFL_FP64
    t0 = time.time()
    h = ifl.prepare_mesh(mesh, ifl.IFL_VERTEX_SCALAR, 1, precision=precision, batch=args.batch, device=0,
                         graphs=0 if args.no_graphs else 1)
    log(f"prepare {time.time() - t0:.1f}s, dofs={h.num_dofs}")
    tune = None
    if not args.no_autotune and args.batch != 1:
        t0 = time.time()
        tune = h.autotune()
        log(f"autotune {time.time() - t0:.2f}s: {tune}")
    fields = torch.from_numpy(fields_h).to(dev)
    fb = max(1, min(args.fields, args.field_block))
    out = torch.zeros((fb, ks.size, h.field_length), dtype=torch.float64, device=dev)
    n_solves = args.fields * ks.size

    agg = {"max_it": 0, "refinements": 0, "solves": 0}

    def step(profile: bool, batch: int = args.batch, prec: int = precision, n_fields: int = args.fields):
        h.set_options(precision=prec, batch=batch, profile=int(profile))
        iters = 0
        for f0 in range(0, n_fields, fb):
            nf = min(fb, n_fields - f0)
            _, st = h.filter(fields[f0:f0 + nf], ks, out=out[:nf])
            iters += sum(s.iterations for s in st)
            if profile:
                agg["max_it"] = max(agg["max_it"], max(s.iterations for s in st))
                agg["refinements"] += sum(s.refinements for s in st)
                agg["solves"] += len(st)
        return iters

    for w in range(args.warmup):
        t = time.time()
        it = step(False)
        torch.cuda.synchronize()
        log(f"warmup {w}: {time.time() - t:.2f}s, {it} CG iterations")
    h.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_it = 0
    for k in range(args.steps):
        total_it += step(True)
        log(f"step {k} done")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    launches, ms, bytes_per = h.profile_read(reset=True)
    mean_s = ms / 1e3 / max(1, launches)
    achieved = bytes_per / mean_s / 1e9 if launches else 0.0
    kernel = h.profile_kernel()
    default_workload = (args.level, args.mask, args.fields, args.scales) == (9, 0.4, 64, 30)
    traffic = recorded_traffic(kernel) if default_workload else None
    value = n_solves * args.steps / el
    res = {
        "metric": "filter solves/s + SpMV HBM GB/s at 2.6M verts; served p50/p99 latency",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if precision == ifl.IFL_MIXED else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"icosphere-L{args.level} {mesh.n_vertices} vertices, {int(args.mask * 100)}% land mask, "
                        f"{args.fields} k^-3 fields x {ks.size} scales, n=1",
            "vertices": mesh.n_vertices,
            "dofs": h.num_dofs,
            "solves_per_step": n_solves,
            "precision": args.precision,
            "batch": args.batch if args.batch else (f"autotuned ({tune['batch']})" if tune else "auto (32)"),
            "autotune": tune,
            "graphs": not args.no_graphs,
            "rtol": 1e-12,
            "mean_cg_iterations": round(total_it / (n_solves * args.steps), 2),
            "max_cg_iterations": agg["max_it"],
            "mean_fp64_replacements": round(agg["refinements"] / max(1, agg["solves"]), 2),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": round(traffic) if traffic else None,
            "kernel": kernel,
            "launches": launches,
            "mean_launch_us": round(mean_s * 1e6, 3),
            "bytes_per_launch": bytes_per,
        },
    }
    if args.plain_fields > 0:
        # the plain FP64 path, one column at a time, on a subset of the fields
        torch.cuda.synchronize()
        t = time.perf_counter()
        it = step(False, batch=1, prec=ifl.IFL_FP64, n_fields=args.plain_fields)
        torch.cuda.synchronize()
        el_p = time.perf_counter() - t
        res["plain_fp64_single_column"] = {
            "value": round(args.plain_fields * ks.size / el_p, 3),
            "unit": "solves/s",
            "sample": f"{args.plain_fields} fields x {ks.size} scales, FP64, one column per solve",
            "mean_cg_iterations": round(it / (args.plain_fields * ks.size), 2),
        }
        res["speedup_vs_plain_fp64"] = round(value / res["plain_fp64_single_column"]["value"], 3)
    # field 0 at every scale in the benchmark's launch configuration, for the
    # parity check on the CPU baseline's sample (not timed)
    h.set_options(precision=precision, batch=args.batch, profile=0)
    h.filter(fields[0:1], ks, out=out[:1])
    torch.cuda.synchronize()
    h.close()
    # the practical streaming rate of this GPU: the library's own copy probe
    # (4 GiB, 16 bytes per thread, one pass), best of 10
    best, med = ifl.stream_probe(0, 4096, 10)
    res["roofline"]["copy_probe_GBs"] = round(best, 1)
    res["roofline"]["copy_probe_median_GBs"] = round(med, 1)
    res["roofline"]["frac_of_copy"] = round(achieved / best, 4)
    # the legs below are reported on their own: a library error in one of
    # them is recorded in its place instead of losing the whole line
    if not args.no_spmv_leg:
        log("SpMV leg on the unmasked level-9 mesh ...")
        try:
            res["spmv_2.6M_vertices"] = spmv_leg(ifl)
        except ifl.IflError as e:
            res["spmv_2.6M_vertices"] = {"error": str(e)}
        log(f"spmv: {res['spmv_2.6M_vertices']}")
    if not args.no_c1c2:
        for name, fn in (("c1_planar_64x64", c1_leg), ("c2_level8_biharmonic", c2_leg),
                         ("orders_reach_64x64", reach_leg)):
            log(f"{name} leg ...")
            try:
                res[name] = fn(ifl)
            except ifl.IflError as e:
                res[name] = {"error": str(e)}
            log(f"{name}: {res[name]}")
    if not args.no_vector_leg:
        log("velocity leg on the level-8 mesh ...")
        try:
            res["velocity_level8"] = vector_leg(ifl)
        except ifl.IflError as e:
            res["velocity_level8"] = {"error": str(e)}
        log(f"velocity: {res['velocity_level8']}")
    if not args.no_serve:
        log("serving leg ...")
        try:
            res["serving"] = serve_leg(args, ifl)
        except (ifl.IflError, RuntimeError) as e:
            res["serving"] = {"error": str(e)}
        log(f"serving: {res['serving']}")
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        parity, res["cpu_baseline"] = cpu_baseline(mesh, fields_h, ks, args.cpu_budget,
                                                   gpu_column=lambda j: out[0, j].cpu().numpy())
        res["parity_sample"] = parity
        workers = args.cpu_workers or min(16, os.cpu_count() or 1)
        if workers > 1:
            log(f"timing the CPU oracle on {workers} worker processes ...")
            one = res["cpu_baseline"]
            rate, done = cpu_parallel(args.level, args.mask, fields_h[0], ks, args.cpu_budget, workers)
            res["cpu_baseline"] = {
                "value": rate, "unit": "solves/s", "cores": workers, "kind": "oracle",
                "sample": f"{done} solves of field 0 spread over {workers} single-threaded worker processes (one per "
                          f"core, each building the oracle's operator first, not counted), ~{args.cpu_budget:g}s each, "
                          f"same mesh and scales as the single-thread figure",
                "single_thread": one,
            }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
