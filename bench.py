#!/usr/bin/env python3
"""Benchmark: particle-neighbour interactions/s of the Eulerian SPH hot path.

Headline workload: 3-D Taylor-Green vortex, 200^3 = 8,000,000 particles in
the periodic unit cube, h = 1.3 dx, c = 10, nu = 0.01, Heun (RK2) steps with
fixed dt (the workload runs 200).  One step = two evaluations of the
corrected Riemann-flux RHS over every directed neighbour pair.  The primary
line is the truncated kernel (cut-off 1.6h); the standard kernel (2h) runs
the same steps for the speed ratio, and both report the kinetic-energy decay
rate at t = 0 against its exact value 24 pi^2 nu (the initial field is an
eigenfunction of the Laplacian).

Printed: ONE JSON line, with
  roofline      the dominant kernel (the 3-D Heun stage kernel) against HBM,
                its VALU issue fraction from the counter profile beside it,
  cpu_baseline  the FP64 oracle on the host cores over bounded samples of the
                3-D workload (headline), the plate and the relaxation,
and further sections: the 2-D Taylor-Green 512^2 (the workload's 1000
steps), the total-Lagrangian plate, the double shear layer, the compressible
rows, the error analysis and the relaxation warm start.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-neighbour interactions/s, 1.6h vs 2h; relax time-to-residue, MLP vs plain"
HBM_PEAK_GBS = 8000.0


# HBM traffic per launch of the stage kernel measured with rocprofv3
# (FETCH_SIZE x 2 + WRITE_SIZE x 1, the factors read off a plain 256 MiB copy),
# keyed by the SHA-256 of the code of the stage kernel's sources (comments and
# blank lines dropped; the stage kernels, the shared header and the window
# builder) it was measured on: a changed kernel reports null until
# it is measured again.  {sha: {"2d": bytes, "3d": bytes}}
# (profiles/euler_heun_stage_taylor_green_2d_512.md and _3d_200.md)
TRAFFIC = {
    "9099615b348286075caa4b1f498fe7bc3e8d5954c9db140060b5023f3dbdce51": {"2d": 39154605, "3d": 1992793621},
}


# VALU wave instructions per launch of the stage kernel (rocprofv3 --pmc
# SQ_INSTS_VALU), keyed like TRAFFIC.  The issue fraction is insts x 4 cycles
# (a wave64 VALU instruction occupies a 16-lane SIMD for 4 cycles) over
# 1,024 SIMDs x 2.4 GHz x the live launch time.
VALU = {
    "9099615b348286075caa4b1f498fe7bc3e8d5954c9db140060b5023f3dbdce51": {"3d": 400299834},
}
VALU_SIMDS = 1024
VALU_CLOCK_HZ = 2.4e9


def _code_lines(text: str):
    """The lines of a C++ source without // comments, trailing blanks and
    empty lines (string literals are kept whole)."""
    out = []
    for line in text.splitlines():
        keep, in_str, k = [], False, 0
        while k < len(line):
            ch = line[k]
            if in_str:
                keep.append(ch)
                if ch == "\\" and k + 1 < len(line):
                    keep.append(line[k + 1])
                    k += 1
                elif ch == '"':
                    in_str = False
            elif ch == '"':
                in_str = True
                keep.append(ch)
            elif line.startswith("//", k):
                break
            else:
                keep.append(ch)
            k += 1
        code = "".join(keep).rstrip()
        if code:
            out.append(code)
    return out


def source_sha(*rels: str) -> str:
    """SHA-256 of the code (comments and blank lines dropped) of the given
    sources, in order."""
    import hashlib
    h = hashlib.sha256()
    for rel in rels:
        with open(os.path.join(ROOT, rel)) as f:
            h.update("\n".join(_code_lines(f.read())).encode())
        h.update(b"\0")
    return h.hexdigest()


STAGE_SOURCES = ("paper_2405_05155_amd/csrc/sph_euler.hip", "paper_2405_05155_amd/csrc/sph_internal.h",
                 "paper_2405_05155_amd/csrc/sph_windows.hip")


def stage_bytes_3d(n: int, nnz: int) -> float:
    """Algorithmic HBM bytes of one RHS evaluation in 3-D: per particle read
    the position (12 B), V (4 B), density (4 B), velocity (12 B) and B
    (36 B), write the four rates (16 B) and read the row offset (8 B): 92 B;
    per neighbour pair the column index (4 B)."""
    return 92.0 * n + 4.0 * nnz


def stage_bytes_2d(n: int, nnz: int) -> float:
    """Algorithmic HBM bytes of one RHS evaluation in 2-D: per particle read
    the position (8 B), V (4 B), density (4 B), velocity (8 B) and the
    correction matrix (16 B), write the three rates (12 B) and read the row
    offset (8 B): 60 B; per neighbour pair the column index (4 B).
    Neighbour records are re-reads served by caches and are not counted."""
    return 60.0 * n + 4.0 * nnz


def run_gpu(w, kappa, steps, warmup, tgv=True):
    import torch

    from paper_2405_05155_amd import sph as S
    f = w.fields
    ctx = S.Context(2)
    ctx.build_cells(S.Domain(dim=2, h=w.h, kappa=kappa), torch.as_tensor(w.pos, device="cuda"))
    ctx.neighbors()
    vol = torch.as_tensor(w.vol, device="cuda")
    ctx.correction_B(vol)
    prm = S.euler_params(c=f["c"], rho0=f["rho0_eos"], rho_ref=f["rho_ref"], eta=f["eta"], mu=f["mu"],
                         dt=w.meta["dt"])
    d = torch.as_tensor(f["drho"], device="cuda").clone()
    m = torch.as_tensor(f["mom"], device="cuda").clone()
    if warmup > 0:
        ctx.euler_step(prm, d, m, warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.euler_step(prm, d, m, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    nnz = ctx.nnz
    ctx.close()
    out = {"ms": ms, "nnz": nnz, "ms_per_step": ms / steps, "launches": 2 * steps,
           "interactions_per_s": 2.0 * nnz * steps / (ms * 1e-3)}
    if tgv:
        out["vel_l2_err"] = tgv_velocity_error(w, d, m, (warmup + steps) * w.meta["dt"])
    return out


def run_gpu_plain(w, kappa, steps, warmup):
    """run_gpu without the Taylor-Green error (any 2-D periodic workload)."""
    return run_gpu(w, kappa, steps, warmup, tgv=False)


def tgv_velocity_error(w, drho, mom, t):
    """Normwise relative L2 error of the velocity against the decaying 2-D
    Taylor-Green solution u0 exp(-8 pi^2 nu t) (not timed)."""
    import numpy as np
    rho = 1.0 + drho.double().cpu().numpy()
    u = mom.double().cpu().numpy() / rho
    x = w.pos.astype(np.float64)
    decay = np.exp(-8.0 * np.pi ** 2 * w.fields["nu"] * t)
    ue = decay * np.stack([np.sin(2 * np.pi * x[0]) * np.cos(2 * np.pi * x[1]),
                           -np.cos(2 * np.pi * x[0]) * np.sin(2 * np.pi * x[1])])
    return float(np.linalg.norm(u - ue) / np.linalg.norm(ue))


def run_shear(nside, kappa, t_marks=(0.8, 1.2)):
    """Double shear layer (Sec. 4.2) from t = 0 to each of t_marks: time per
    Heun step (HIP events over the whole run) and, at each mark, the
    velocity field and the kinetic energy (not timed)."""
    import numpy as np
    import torch

    from paper_2405_05155_amd import inputs as I
    from paper_2405_05155_amd import sph as S
    w = I.double_shear_layer(nside=nside)
    f = w.fields
    ctx = S.Context(2)
    ctx.build_cells(S.Domain(dim=2, h=w.h, kappa=kappa), torch.as_tensor(w.pos, device="cuda"))
    ctx.neighbors()
    ctx.correction_B(torch.as_tensor(w.vol, device="cuda"))
    dt = w.meta["dt"]
    prm = S.euler_params(c=f["c"], rho0=f["rho0_eos"], rho_ref=f["rho_ref"], eta=f["eta"], mu=f["mu"], dt=dt)
    d = torch.as_tensor(f["drho"], device="cuda").clone()
    m = torch.as_tensor(f["mom"], device="cuda").clone()
    vol = w.vol.astype(np.float64)

    def energy_and_velocity():
        rho = 1.0 + d.double().cpu().numpy()
        u = m.double().cpu().numpy() / rho
        return float(0.5 * np.sum(rho * (u ** 2).sum(0) * vol)), u

    ke0, _ = energy_and_velocity()
    # untimed warm-up on copies (first launches, row preparation)
    ctx.euler_step(prm, d.clone(), m.clone(), 5)
    stream = torch.cuda.current_stream()
    done, ms, marks = 0, 0.0, []
    for t in t_marks:
        steps = int(round(t / dt)) - done
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.euler_step(prm, d, m, steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms += e0.elapsed_time(e1)
        done += steps
        ke, u = energy_and_velocity()
        marks.append({"t": done * dt, "ke_over_ke0": ke / ke0, "u": u})
    nnz = ctx.nnz
    ctx.close()
    return {"n_particles": w.n, "nnz": nnz, "steps": done, "ms_per_step": ms / done,
            "interactions_per_s": 2.0 * nnz * done / (ms * 1e-3), "marks": marks}


def shear_layer_section(nside=128, nside_big=1024, steps_big=400):
    """TW against SW on the double shear layer: the paper's resolution run
    to t = 0.8 and 1.2 (time per step, kinetic energy, velocity difference
    between the two runs), and the time per step at nside_big^2."""
    import numpy as np
    from paper_2405_05155_amd import inputs as I
    tw, sw = run_shear(nside, 1.6), run_shear(nside, 2.0)
    out = {"nside": nside, "steps": tw["steps"], "ms_per_step_tw": tw["ms_per_step"],
           "ms_per_step_sw": sw["ms_per_step"], "alpha_gpu": tw["ms_per_step"] / sw["ms_per_step"],
           "alpha_paper_cpu": 17.83 / 29.99, "marks": []}
    for a, b in zip(tw["marks"], sw["marks"]):
        out["marks"].append({"t": a["t"], "ke_over_ke0_tw": a["ke_over_ke0"], "ke_over_ke0_sw": b["ke_over_ke0"],
                             "vel_rel_diff_tw_sw": float(np.linalg.norm(a["u"] - b["u"]) / np.linalg.norm(b["u"]))})
    w = I.double_shear_layer(nside=nside_big)
    big = {k: run_gpu_plain(w, k, steps_big, 10) for k in (1.6, 2.0)}
    out["large"] = {"nside": nside_big, "steps": steps_big, "ms_per_step_tw": big[1.6]["ms_per_step"],
                    "ms_per_step_sw": big[2.0]["ms_per_step"],
                    "alpha_gpu": big[1.6]["ms_per_step"] / big[2.0]["ms_per_step"],
                    "interactions_per_s_tw": big[1.6]["interactions_per_s"]}
    return out


def run_hllc(nside, kappa, t_end=0.25):
    """Compressible rows (limited HLLC, ideal gas) on the advected density
    wave: time per Heun step over the run to t_end (HIP events, after an
    untimed warm-up on copies) and the density error against the exact
    shifted profile (not timed)."""
    import numpy as np
    import torch

    from paper_2405_05155_amd import inputs as I
    from paper_2405_05155_amd import sph as S
    w = I.density_wave_2d(nside=nside)
    f = w.fields
    ctx = S.Context(2)
    ctx.build_cells(S.Domain(dim=2, h=w.h, kappa=kappa), torch.as_tensor(w.pos, device="cuda"))
    ctx.neighbors()
    ctx.correction_B(torch.as_tensor(w.vol, device="cuda"))
    dt = w.meta["dt"]
    prm = S.hllc_params(f["gamma"], f["eta"], dt)
    r = torch.as_tensor(f["rho"], device="cuda").clone()
    m = torch.as_tensor(f["mom"], device="cuda").clone()
    e = torch.as_tensor(f["E"], device="cuda").clone()
    ctx.hllc_step(prm, r.clone(), m.clone(), e.clone(), 5)
    steps = int(round(t_end / dt))
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.hllc_step(prm, r, m, e, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    nnz = ctx.nnz
    ctx.close()
    x = w.pos[0].astype(np.float64)
    t = steps * dt
    exact = 1.0 + f["amplitude"] * np.sin(2 * np.pi * (x - f["U"] * t))
    rho = r.double().cpu().numpy()
    return {"n_particles": w.n, "nnz": nnz, "steps": steps, "ms_per_step": ms / steps,
            "interactions_per_s": 2.0 * nnz * steps / (ms * 1e-3),
            "density_rel_l2_err": float(np.linalg.norm(rho - exact) / np.linalg.norm(exact - 1.0))}


def sod_error(kappa, nx=512):
    """Sod's shock tube in a periodic strip (nx x 16) to t = 0.1 on the GPU:
    mean density error on [1/2, 1) against the exact solution (not timed)."""
    import numpy as np
    import torch

    from paper_2405_05155_amd import inputs as I
    from paper_2405_05155_amd import sph as S
    from paper_2405_05155_amd.exact import sod_density
    w = I.sod_strip_2d(nx)
    f = w.fields
    ctx = S.Context(2)
    ctx.build_cells(S.Domain(dim=2, h=w.h, kappa=kappa, lo=w.lo, hi=w.hi, periodic=w.periodic),
                    torch.as_tensor(w.pos, device="cuda"))
    ctx.correction_B(torch.as_tensor(w.vol, device="cuda"))
    dt = w.meta["dt"]
    steps = int(round(0.1 / dt))
    r = torch.as_tensor(f["rho"], device="cuda").clone()
    m = torch.as_tensor(f["mom"], device="cuda").clone()
    e = torch.as_tensor(f["E"], device="cuda").clone()
    ctx.hllc_step(S.hllc_params(f["gamma"], f["eta"], dt), r, m, e, steps)
    rho = r.double().cpu().numpy()
    ctx.close()
    x = w.pos[0].astype(np.float64)
    sel = x >= 0.5
    exact = np.array([sod_density((xx - 0.75) / (steps * dt)) for xx in x[sel]])
    return float(np.mean(np.abs(rho[sel] - exact)))


def compressible_section(nside=512):
    tw, sw = run_hllc(nside, 1.6), run_hllc(nside, 2.0)
    sod_tw, sod_sw = sod_error(1.6), sod_error(2.0)
    return {"workload": f"density_wave_2d_{nside} (ideal gas, limited HLLC, a quarter period)",
            "kappa1.6": tw, "kappa2": sw, "speedup_tw_over_sw": sw["ms_per_step"] / tw["ms_per_step"],
            "err_ratio_tw_over_sw": tw["density_rel_l2_err"] / sw["density_rel_l2_err"],
            "sod_512x16_t0.1": {"mean_density_err_tw": sod_tw, "mean_density_err_sw": sod_sw,
                                "reference": "exact Riemann solution"}}


def error_analysis_section():
    """Sec. 2.3.3 through the GPU's gradient: on the lattice (Fig. 2, upper
    panel) the L2 error of df/dx, f = exp(-x^2/0.1), at dp = D/10, D/20, D/40
    with and without the correction and the observed orders; then the same
    on the circle relaxed on the GPU with the LG and with the Wendland
    kernel (the two lower panels) and Table 1's relaxed rows."""
    import math

    import numpy as np
    import torch

    from paper_2405_05155_amd import inputs as I
    from paper_2405_05155_amd import sph as S
    out = {"function": "f = exp(-x^2/0.1), D = 2, h = 1.3 dp, lattice", "dp": ["D/10", "D/20", "D/40"]}
    for kappa, tag in ((2.0, "SW"), (1.6, "TW")):
        for corrected in (False, True):
            errs = []
            for nside in (10, 20, 40):
                w = I.gradient_lattice_2d(nside)
                ctx = S.Context(2)
                ctx.build_cells(S.Domain(dim=2, h=w.h, kappa=kappa, lo=w.lo, hi=w.hi, periodic=w.periodic),
                                torch.as_tensor(w.pos, device="cuda"))
                vol = torch.as_tensor(w.vol, device="cuda")
                if corrected:
                    ctx.correction_B(vol)
                else:
                    ctx.set_correction(vol, torch.eye(2, device="cuda").repeat(w.n, 1, 1).contiguous())
                g = ctx.gradient(torch.as_tensor(w.fields["f"], device="cuda"))[0].double().cpu().numpy()
                ctx.close()
                ex = w.fields["dfdx"]
                errs.append(float(np.linalg.norm(g - ex) / np.linalg.norm(ex)))
            out[f"{tag} {'with' if corrected else 'without'} B"] = {
                "l2": errs, "orders": [math.log2(errs[i] / errs[i + 1]) for i in range(2)]}
    out["lg_relaxed_circle"] = relaxed_circle_errors()
    out["wendland_relaxed_circle"] = relaxed_circle_errors(kernel="Wendland")
    return out


def relaxed_circle_errors(ndivs=(10, 20, 40), kernel="LG", iters=400):
    """Fig. 2's relaxed panels and Table 1's relaxed rows on the paper's 2-D
    circle (D = 2, dp = D/10, D/20, D/40): the seed-2 fill relaxed on the GPU
    (LG: to R < 1e-4, the residue checked every 10 iterations; Wendland:
    `iters` iterations), then the GPU's gradient of f = exp(-x^2/0.1) with
    and without the correction over every particle (L2 error of df/dx and
    the observed orders), and at D/10 the kernel-sum error (f = 1, no
    correction) over the particles whose support lies inside the circle."""
    import math

    import numpy as np
    import torch

    from paper_2405_05155_amd import inputs as I
    from paper_2405_05155_amd import sph as S
    errs, residues, table1, its = {}, [], {}, []
    for nd in ndivs:
        w = I.circle_fill(dx=2.0 / nd, seed=2)
        f0 = w.fields
        dom = S.Domain(dim=2, h=w.h, kappa=2.0, lo=w.lo, hi=w.hi, periodic=(0, 0), kernel=S.LAGUERRE_GAUSS)
        prm = S.relax_params(f0["center"], f0["radius"], p0=f0["p0"], rho=f0["rho"],
                             kernel=S.LAGUERRE_GAUSS if kernel == "LG" else S.WENDLAND)
        rctx = S.Context(2)
        vol = torch.as_tensor(w.vol, device="cuda")
        pos = torch.as_tensor(w.pos, device="cuda").clone()
        u = torch.zeros_like(pos)
        res = torch.zeros(1, dtype=torch.float64, device="cuda")
        done = 0
        while done < (3000 if kernel == "LG" else iters):
            r, _ = rctx.relax_residue(dom, prm, pos, vol, want_g=False)
            if kernel == "LG" and float(r.item()) < 1e-4:
                break
            rctx.relax_step(dom, prm, pos, u, vol, 10, res)
            done += 10
        r, _ = rctx.relax_residue(dom, prm, pos, vol, want_g=False)
        residues.append(float(r.item()))
        its.append(done)
        rctx.close()
        p = pos.cpu().numpy()
        f, ex = I.circle_gradient_fields(p)
        inner = np.sqrt((p.astype(np.float64) ** 2).sum(0)) < f0["radius"] - 2.0 * w.h
        for kappa, tag in ((2.0, "SW"), (1.6, "TW")):
            ctx = S.Context(2)
            ctx.build_cells(S.Domain(dim=2, h=w.h, kappa=kappa, lo=w.lo, hi=w.hi, periodic=(0, 0)), pos)
            if nd == ndivs[0]:
                ks = ctx.kernel_sum(vol).double().cpu().numpy()[inner]
                table1[tag] = math.sqrt(float(np.mean((ks - 1.0) ** 2)))   # Eq. (10), phi = 1
                table1["interior_particles"] = int(inner.sum())
            for corrected in (False, True):
                if corrected:
                    ctx.correction_B(vol)
                else:
                    ctx.set_correction(vol, torch.eye(2, device="cuda").repeat(w.n, 1, 1).contiguous())
                g = ctx.gradient(torch.as_tensor(f.astype(np.float32), device="cuda"))[0].double().cpu().numpy()
                errs.setdefault(f"{tag} {'with' if corrected else 'without'} B", []).append(
                    float(np.linalg.norm(g - ex) / np.linalg.norm(ex)))
            ctx.close()
    out = {"dp": [f"D/{k}" for k in ndivs], "diameter": 2.0, "relaxation": kernel, "iterations": its,
           "final_residue": residues}
    for k, v in errs.items():
        out[k] = {"l2": v, "orders": [math.log2(v[i] / v[i + 1]) for i in range(len(v) - 1)]}
    printed = {"LG": [0.037, 0.031], "Wendland": [0.034, 0.028]}[kernel]
    out["table1_kernel_sum"] = dict(table1, dp=f"D/{ndivs[0]}", printed_sw_tw=printed)
    return out


def _ke(vol, drho, mom, rho_ref=1.0):
    """Kinetic energy sum_i V_i |m_i|^2 / (2 rho_i) of a device state (FP64)."""
    rho = rho_ref + drho.double()
    return float((vol.double() * (mom.double() ** 2).sum(0) / (2.0 * rho)).sum())


def run_euler_3d(nside, kappa, steps, warmup, accuracy_steps=0):
    """3-D Taylor-Green in the periodic unit cube (nside^3 particles): time
    per Heun step over `steps` steps after `warmup` untimed ones (HIP events
    on the context's stream); the kinetic-energy decay rate at t = 0 from
    the RHS; with accuracy_steps > warmup + steps the run continues untimed
    to accuracy_steps, and the final velocity and kinetic energy are
    returned (not timed)."""
    import torch

    from paper_2405_05155_amd import inputs as I
    from paper_2405_05155_amd import sph as S
    w = I.taylor_green_3d(nside=nside)
    f = w.fields
    ctx = S.Context(3)
    ctx.build_cells(S.Domain(dim=3, h=w.h, kappa=kappa), torch.as_tensor(w.pos, device="cuda"))
    ctx.neighbors()
    vol = torch.as_tensor(w.vol, device="cuda")
    ctx.correction_B(vol)
    prm = S.euler_params(c=f["c"], rho0=f["rho0_eos"], rho_ref=f["rho_ref"], eta=f["eta"], mu=f["mu"],
                         dt=w.meta["dt"])
    d = torch.as_tensor(f["drho"], device="cuda").clone()
    m = torch.as_tensor(f["mom"], device="cuda").clone()
    # kinetic-energy rate at t = 0: dK/dt = sum V (m . dm/dt / rho - |m|^2 drho/dt / (2 rho^2))
    dr, dm = ctx.euler_rhs(prm, d, m)
    rho = f["rho_ref"] + d.double()
    m2 = (m.double() ** 2).sum(0)
    dK = float((vol.double() * ((m.double() * dm.double()).sum(0) / rho - m2 * dr.double() / (2 * rho ** 2))).sum())
    ke0 = _ke(vol, d, m, f["rho_ref"])
    del dr, dm, rho, m2
    if warmup > 0:
        ctx.euler_step(prm, d, m, warmup)
    stream = ctx.stream
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.euler_step(prm, d, m, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    nnz = ctx.nnz
    out = {"n_particles": w.n, "nnz": nnz, "steps": steps, "ms_per_step": ms / steps,
           "interactions_per_s": 2.0 * nnz * steps / (ms * 1e-3)}
    launch_s = ms * 1e-3 / (2 * steps)
    bytes_launch = stage_bytes_3d(w.n, nnz)
    out.update({"avg_launch_us": launch_s * 1e6, "bytes_per_launch": bytes_launch,
                "achieved_GBs": bytes_launch / launch_s / 1e9, "ke_rate_t0": -dK / ke0, "dt": w.meta["dt"]})
    done = warmup + steps
    if accuracy_steps > done:
        ctx.euler_step(prm, d, m, accuracy_steps - done)
        done = accuracy_steps
    out["t_end"] = done * w.meta["dt"]
    out["ke_end_over_ke0"] = _ke(vol, d, m, f["rho_ref"]) / ke0
    out["_vel"] = m.double() / (f["rho_ref"] + d.double())
    ctx.close()
    return out


def tgv3d_accuracy(tw, sw, nu):
    """Accuracy of the two 3-D runs: the kinetic-energy decay rate at t = 0
    against 24 pi^2 nu (exact for the initial field), the energy at the end
    of the run against the first-order estimate exp(-24 pi^2 nu t), and the
    relative L2 difference of the two final velocity fields."""
    import math
    exact = 24.0 * math.pi ** 2 * nu
    e_tw, e_sw = abs(tw["ke_rate_t0"] / exact - 1.0), abs(sw["ke_rate_t0"] / exact - 1.0)
    diff = float((tw["_vel"] - sw["_vel"]).norm() / sw["_vel"].norm())
    return {"ke_decay_rate_t0": {"exact_24pi2nu": exact, "tw": tw["ke_rate_t0"], "sw": sw["ke_rate_t0"],
                                 "rel_err_tw": e_tw, "rel_err_sw": e_sw, "err_ratio_tw_over_sw": e_tw / e_sw},
            "run": {"t": tw["t_end"], "ke_over_ke0_tw": tw["ke_end_over_ke0"], "ke_over_ke0_sw": sw["ke_end_over_ke0"],
                    "exp_minus_24pi2nu_t": math.exp(-exact * tw["t_end"]), "vel_rel_diff_tw_sw": diff},
            "viscous_term": "2 mu sum_j V_j c_ij (v_i - v_j) W'/r, c_ij = (tr B_i + tr B_j)/(2d)"}


def run_plate(kappa, steps, warmup, nx=430):
    """TLSPH cantilever plate 0.2 x 0.02 x 0.04 at dx = 0.2/nx (plus four
    clamp layers), neo-Hookean, kick-drift-kick steps."""
    import torch

    from paper_2405_05155_amd import inputs as I
    from paper_2405_05155_amd import sph as S
    w = I.cantilever_plate(nx=nx)
    f = w.fields
    ctx = S.Context(3)
    ctx.build_cells(S.Domain(dim=3, h=w.h, kappa=kappa, lo=w.lo, hi=w.hi, periodic=(0, 0, 0)),
                    torch.as_tensor(w.pos, device="cuda"))
    ctx.neighbors()
    ctx.correction_B(torch.as_tensor(w.vol, device="cuda"))
    prm = S.tlsph_params(f["rho0"], f["E"], f["nu"], dt=w.meta["dt"], model=0)
    pos = torch.as_tensor(w.pos, device="cuda").clone()
    vel = torch.as_tensor(w.fields["vel"], device="cuda").clone()
    F = torch.eye(3, device="cuda").repeat(w.n, 1, 1).contiguous()
    fixed = torch.as_tensor(f["fixed"], device="cuda")
    _, acc = ctx.tlsph_rhs(prm, vel, F, fixed)
    ctx.tlsph_step(prm, fixed, pos, vel, F, acc, warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ctx.tlsph_step(prm, fixed, pos, vel, F, acc, steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    nnz = ctx.nnz
    ctx.close()
    return {"n_particles": w.n, "nnz": nnz, "ms_per_step": ms / steps,
            "interactions_per_s": 2.0 * nnz * steps / (ms * 1e-3)}


def plate_tip_history(kappa, steps, every, nx=430):
    """Tip deflection (mean y displacement of the free-end layer) of the
    cantilever plate every `every` kick-drift-kick steps (not timed)."""
    import numpy as np
    import torch

    from paper_2405_05155_amd import inputs as I
    from paper_2405_05155_amd import sph as S
    w = I.cantilever_plate(nx=nx)
    f = w.fields
    ctx = S.Context(3)
    ctx.build_cells(S.Domain(dim=3, h=w.h, kappa=kappa, lo=w.lo, hi=w.hi, periodic=(0, 0, 0)),
                    torch.as_tensor(w.pos, device="cuda"))
    ctx.correction_B(torch.as_tensor(w.vol, device="cuda"))
    prm = S.tlsph_params(f["rho0"], f["E"], f["nu"], dt=w.meta["dt"], model=0)
    pos = torch.as_tensor(w.pos, device="cuda").clone()
    y0 = pos[1].clone()
    vel = torch.as_tensor(f["vel"], device="cuda").clone()
    F = torch.eye(3, device="cuda").repeat(w.n, 1, 1).contiguous()
    fixed = torch.as_tensor(f["fixed"], device="cuda")
    xmax = float(w.pos[0].max())
    tip = torch.as_tensor(w.pos[0] > xmax - 0.5 * w.meta["dx"], device="cuda")
    _, acc = ctx.tlsph_rhs(prm, vel, F, fixed)
    hist = []
    for _ in range(steps // every):
        ctx.tlsph_step(prm, fixed, pos, vel, F, acc, every)
        hist.append(float((pos[1] - y0)[tip].double().mean()))
    ctx.close()
    return np.array(hist)


def host_cpu():
    """Model name and logical CPU count of the host the oracle runs on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count()}


def run_cpu_baseline(w, kappa, budget_s):
    """The FP64 oracle on a 2-D Taylor-Green workload: Heun steps timed
    until the budget is spent (neighbours and B not timed)."""
    import numpy as np

    import oracle as O
    f = w.fields
    box = O.make_box(2)
    rc = kappa * w.h
    rp, col = O.neighbors_grid(box, w.pos, rc, rc * rc)
    B, _ = O.correction_B(box, w.pos, O.WENDLAND, w.h, rp, col, w.vol)
    prm = O.euler_params(c=f["c"], rho0=f["rho0_eos"], eta=f["eta"], mu=f["mu"], dt=w.meta["dt"])
    rho = f["rho_ref"] + f["drho"].astype(np.float64)
    mom = f["mom"].astype(np.float64)
    t0 = time.perf_counter()
    rho, mom = O.euler_heun(box, w.pos, w.h, rp, col, w.vol, B, prm, rho, mom, 1)
    t1 = time.perf_counter() - t0
    steps = max(1, min(200, int(budget_s / max(t1, 1e-6))))
    t0 = time.perf_counter()
    O.euler_heun(box, w.pos, w.h, rp, col, w.vol, B, prm, rho, mom, steps)
    dt = time.perf_counter() - t0
    nnz = int(rp[-1])
    side = int(round(w.n ** 0.5))
    return {"value": 2.0 * nnz * steps / dt, "unit": "interactions/s", "cores": O.num_threads(), "kind": "oracle",
            "ms_per_step": dt * 1e3 / steps,
            "sample": f"{steps} Heun steps of the 2-D Taylor-Green {side}^2 workload at kappa={kappa} "
                      f"(FP64 oracle, {dt:.1f} s)"}


def run_cpu_3d(budget_s, nside=200, kappa=1.6, max_steps=10):
    """The FP64 oracle on the headline workload (3-D Taylor-Green, nside^3):
    neighbour search and B of every particle (set-up, not timed), then the
    first Heun steps from the initial state, timed until the budget is spent
    (at least one, at most max_steps)."""
    import numpy as np

    import oracle as O
    from paper_2405_05155_amd import inputs as I
    w = I.taylor_green_3d(nside=nside)
    f = w.fields
    box = O.make_box(3)
    rc = kappa * w.h
    t0 = time.perf_counter()
    rp, col = O.neighbors_grid(box, w.pos, rc, rc * rc)
    B, _ = O.correction_B(box, w.pos, O.WENDLAND, w.h, rp, col, w.vol)
    setup = time.perf_counter() - t0
    prm = O.euler_params(c=f["c"], rho0=f["rho0_eos"], eta=f["eta"], mu=f["mu"], dt=w.meta["dt"])
    rho = f["rho_ref"] + f["drho"].astype(np.float64)
    mom = f["mom"].astype(np.float64)
    steps, secs = 0, 0.0
    while steps < max_steps and (steps == 0 or secs + secs / steps <= budget_s):
        t0 = time.perf_counter()
        rho, mom = O.euler_heun(box, w.pos, w.h, rp, col, w.vol, B, prm, rho, mom, 1)
        secs += time.perf_counter() - t0
        steps += 1
    nnz = int(rp[-1])
    return {"value": 2.0 * nnz * steps / secs, "unit": "interactions/s", "cores": O.num_threads(), "kind": "oracle",
            "ms_per_step": secs * 1e3 / steps,
            "sample": f"the first {steps} of the 200 Heun steps of the {nside}^3 3-D Taylor-Green workload at "
                      f"kappa={kappa} (FP64 oracle, {secs:.1f} s; neighbour search and B, {setup:.1f} s, not timed)"}


def run_cpu_plate(budget_s, kappa=1.6, nx=430, max_steps=50):
    """The FP64 oracle on the total-Lagrangian plate (1,604,932 particles):
    the first kick-drift-kick steps, timed until the budget is spent."""
    import numpy as np

    import oracle as O
    from paper_2405_05155_amd import inputs as I
    w = I.cantilever_plate(nx=nx)
    f = w.fields
    box = O.make_box(3, lo=w.lo, hi=w.hi, periodic=(0, 0, 0))
    rc = kappa * w.h
    rp, col = O.neighbors_grid(box, w.pos, rc, rc * rc)
    B, _ = O.correction_B(box, w.pos, O.WENDLAND, w.h, rp, col, w.vol)
    prm = O.tlsph_params(f["rho0"], f["E"], f["nu"], dt=w.meta["dt"], model=0)
    F = np.tile(np.eye(3), (w.n, 1, 1))
    pos, vel, fixed = w.pos.astype(np.float64), f["vel"].astype(np.float64), f["fixed"]
    _, acc, _ = O.tlsph_rhs(box, w.pos, w.h, rp, col, w.vol, B, prm, vel, F, fixed)
    steps, secs = 0, 0.0
    while steps < max_steps and (steps == 0 or secs + secs / steps <= budget_s):
        t0 = time.perf_counter()
        pos, vel, F, acc = O.tlsph_step(box, w.pos, w.h, rp, col, w.vol, B, prm, fixed, pos, vel, F, acc, 1)
        secs += time.perf_counter() - t0
        steps += 1
    nnz = int(rp[-1])
    return {"value": 2.0 * nnz * steps / secs, "unit": "interactions/s", "cores": O.num_threads(), "kind": "oracle",
            "ms_per_step": secs * 1e3 / steps,
            "sample": f"the first {steps} of the 2000 kick-drift-kick steps of the {w.n}-particle plate at "
                      f"kappa={kappa} (FP64 oracle, {secs:.1f} s)"}


def run_cpu_relax(budget_s, nside=260, max_iter=200):
    """The FP64 oracle on the relaxation workload (the seed-2 sphere,
    1,987,776 particles at dx = 1/260): the first iterations (each with a
    fresh neighbour search, as on the GPU), timed until the budget is
    spent."""
    import numpy as np

    import oracle as O
    from paper_2405_05155_amd import inputs as I
    w = I.sphere_fill(dx=1.0 / nside, seed=2)
    f = w.fields
    box = O.make_box(3, lo=w.lo, hi=w.hi, periodic=(0, 0, 0))
    prm = O.relax_params(w.h, f["center"], f["radius"], p0=f["p0"], rho=f["rho"])
    pos, u = w.pos.astype(np.float64), np.zeros((3, w.n))
    iters, secs = 0, 0.0
    while iters < max_iter and (iters == 0 or secs + secs / iters <= budget_s):
        t0 = time.perf_counter()
        pos, u, _ = O.relax_run(box, pos, prm, w.vol, 1, u=u)
        secs += time.perf_counter() - t0
        iters += 1
    return {"ms_per_iteration": secs * 1e3 / iters, "cores": O.num_threads(), "kind": "oracle",
            "sample": f"the first {iters} iterations of the {w.n}-particle sphere relaxation "
                      f"(FP64 oracle, {secs:.1f} s)"}


def run_cpu_one_core(kappa, budget_s):
    """The same oracle leg on one host core, in a child process started with
    OMP_NUM_THREADS=1 before this process touches the GPU."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-only-json", "--cpu-budget", str(budget_s),
                        "--kappa", str(kappa)], env=env, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr.strip()[-300:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def run_relax(epochs, nside=260):
    """Relaxation time-to-residue (R < 1e-4), plain vs learned warm start, on
    the sphere of radius 0.3 (dx = 1/nside; 1,987,776 particles at 260).
    The network is trained (not timed) on the plain trajectory of seed 1:
    snapshots every 20 iterations up to 180, targets (r_final - r_k)/h,
    batch 65,536, AdamW lr 1e-3; the timed runs use seed 2."""
    import torch

    from paper_2405_05155_amd import inputs as I
    from paper_2405_05155_amd import sph as S
    from paper_2405_05155_amd import warmstart as WS
    ctx = S.Context(3)
    w1 = I.sphere_fill(dx=1.0 / nside, seed=1)
    run1, final, snaps = WS.relax_plain(ctx, w1, snapshot_every=20, snapshot_until=180)
    feat, targ = WS.training_set(ctx, w1, snaps, final)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    params, losses = WS.train(ctx, feat, targ, epochs=epochs, init=init_params(0))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    var = float(targ.pow(2).mean())
    nsamp = int(feat.shape[0])
    del feat, targ, snaps
    w2 = I.sphere_fill(dx=1.0 / nside, seed=2)
    WS.relax_plain(ctx, w2, max_iter=20)          # warm the code paths
    plain, _, _ = WS.relax_plain(ctx, w2)
    warm, _ = WS.relax_warm(ctx, w2, params)
    return {"metric": "relax time-to-residue (R < 1e-4), MLP warm start vs plain", "n_particles": w2.n,
            "plain_s": plain.seconds, "plain_iters": plain.iterations, "mlp_s": warm.seconds,
            "mlp_iters": warm.iterations, "ratio_mlp_over_plain": warm.seconds / plain.seconds,
            "mlp_moves_accepted": warm.accepted, "mlp_moves_tried": warm.attempted,
            "train_s": train_s, "train_samples": nsamp, "train_epochs": epochs,
            "train_loss_first_last": [losses[0], losses[-1]], "target_mean_square": var,
            "train_trajectory_iters": run1.iterations}


def run_train(steps, batch=65536, nbatch=20):
    """MLP training throughput on a synthetic feature set shaped like the
    relaxation's (nbatch x batch rows of MLP_FEAT_STRIDE BF16 features, the
    first 100 columns N(0, 0.5^2), targets N(0, 0.08^2)): the training loop
    of warmstart.train (shuffle, batch gather, train step) for
    ceil(steps / nbatch) epochs after one warm-up epoch."""
    import torch

    from paper_2405_05155_amd import sph as S
    from paper_2405_05155_amd import warmstart as WS
    ctx = S.Context(3)
    n = batch * nbatch
    g = torch.Generator(device="cpu").manual_seed(5)
    x = torch.zeros((n, S.MLP_FEAT_STRIDE), dtype=torch.float32)
    x[:, :100] = 0.5 * torch.randn((n, 100), generator=g)
    feat = x.to(torch.bfloat16).view(torch.int16).to("cuda")
    targ = (0.08 * torch.randn((n, 3), generator=g)).to("cuda")
    del x
    init = init_params(0)
    WS.train(ctx, feat, targ, epochs=1, batch=batch, init=init)
    epochs = max(1, -(-steps // nbatch))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, losses = WS.train(ctx, feat, targ, epochs=epochs, batch=batch, init=init)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    nstep = epochs * nbatch
    return {"train_steps": nstep, "batch": batch, "ms_per_step": secs * 1e3 / nstep,
            "samples_per_s": nstep * batch / secs, "loss_first_last": [losses[0], losses[-1]]}


def run_setup(reps=5):
    """Set-up path of the fixed-particle workloads (2-D 512^2 and 3-D 200^3
    Taylor-Green, cut-offs 1.6h and 2h): cell binning and neighbour search
    (sph_build_cells), the caller-order neighbour export, the kernel sum and
    the correction matrices; milliseconds per call, best of `reps`."""
    import torch

    from paper_2405_05155_amd import inputs as I
    from paper_2405_05155_amd import sph as S

    def best(fn):
        out = float("inf")
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            out = min(out, (time.perf_counter() - t0) * 1e3)
        return out

    res = {}
    for name, w in (("taylor_green_2d_512", I.taylor_green_2d(nside=512)),
                    ("taylor_green_3d_200", I.taylor_green_3d(nside=200))):
        pos = torch.as_tensor(w.pos, device="cuda")
        vol = torch.as_tensor(w.vol, device="cuda")
        for kappa in (1.6, 2.0):
            ctx = S.Context(w.dim)
            dom = S.Domain(dim=w.dim, h=w.h, kappa=kappa)
            ctx.build_cells(dom, pos)
            r = {"n_particles": w.n, "nnz": ctx.nnz, "build_cells_ms": best(lambda: ctx.build_cells(dom, pos))}
            r["export_ms"] = best(lambda: (ctx.build_cells(dom, pos), ctx.neighbors())) - r["build_cells_ms"]
            r["kernel_sum_ms"] = best(lambda: ctx.kernel_sum(vol))
            r["correction_B_ms"] = best(lambda: ctx.correction_B(vol))
            res[f"{name}_kappa{kappa}"] = r
            ctx.close()
            torch.cuda.empty_cache()
    return res


def init_params(seed):
    """Seeded initial weights U(-1/sqrt(fan_in), 1/sqrt(fan_in)) (PyTorch's
    linear-layer default), drawn on the host and passed in."""
    import numpy as np
    rng = np.random.default_rng(seed)
    shapes = [(128, 100, 100), (128, 0, 100), (128, 128, 128), (128, 0, 128), (3, 128, 128), (3, 0, 128)]
    parts = []
    for rows, cols, fan_in in shapes:
        b = 1.0 / fan_in ** 0.5
        parts.append(rng.uniform(-b, b, size=(rows, cols) if cols else (rows,)).reshape(-1))
    return np.concatenate(parts).astype(np.float32)


def log(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def main():
    import numpy as np
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200,
                    help="timed Heun steps of the 200^3 3-D Taylor-Green headline (the workload runs 200)")
    ap.add_argument("--warmup", type=int, default=10, help="untimed 3-D steps before the timed ones")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="seconds of timed oracle work on the headline workload")
    ap.add_argument("--cpu-budget-extra", type=float, default=5.0,
                    help="seconds of timed oracle work on each of the plate, the relaxation and the 2-D workload")
    ap.add_argument("--nside2d", type=int, default=512)
    ap.add_argument("--steps2d", type=int, default=500,
                    help="timed 2-D Taylor-Green steps, after as many untimed ones (the workload's 1000 in all)")
    ap.add_argument("--no-relax", action="store_true", help="skip the relaxation time-to-residue part")
    ap.add_argument("--relax-epochs", type=int, default=50)
    ap.add_argument("--relax-nside", type=int, default=260)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 2-D, plate, shear-layer, compressible and error-analysis sections")
    ap.add_argument("--nside3d", type=int, default=200)
    ap.add_argument("--steps-plate", type=int, default=2000, help="timed plate steps (the workload runs 2000)")
    ap.add_argument("--plate-accuracy-steps", type=int, default=2000,
                    help="untimed TW-vs-SW tip-deflection history of the plate (0: skip)")
    ap.add_argument("--kappa", type=float, default=0.0, help="profile the 2-D Taylor-Green line only, at this cut-off")
    ap.add_argument("--kappa3d", type=float, default=0.0, help="profile the 3-D Taylor-Green line only, at this cut-off")
    ap.add_argument("--plate", type=float, default=0.0, help="profile the TLSPH plate line only, at this cut-off")
    ap.add_argument("--shear", action="store_true", help="the double shear layer section only")
    ap.add_argument("--compressible", action="store_true", help="the compressible (HLLC) section only")
    ap.add_argument("--error-analysis", action="store_true", help="the error-analysis section only")
    ap.add_argument("--relax-iters", type=int, default=0, help="profile N plain relaxation iterations only")
    ap.add_argument("--train-steps", type=int, default=0, help="profile N MLP training steps only")
    ap.add_argument("--cpu-only-json", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-one-core-budget", type=float, default=3.0,
                    help="seconds of single-core oracle time on the 2-D workload (0: skip)")
    ap.add_argument("--setup", action="store_true", help="profile the set-up path only (binning, neighbours, "
                    "kernel sum, correction matrices)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("multi-GPU runs are not supported: the hot path runs on one GPU; use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.cpu_only_json:  # child of run_cpu_one_core: oracle only, no GPU
        from paper_2405_05155_amd import inputs as I
        print(json.dumps(run_cpu_baseline(I.taylor_green_2d(nside=args.nside2d), args.kappa or 1.6,
                                          args.cpu_budget)))
        return
    one_core = None
    default_run = not (args.kappa or args.relax_iters or args.kappa3d or args.train_steps or args.setup
                       or args.plate or args.shear or args.compressible or args.error_analysis)
    if default_run and not args.no_cpu_baseline and args.cpu_one_core_budget > 0:
        log("oracle on one core (2-D workload)")
        one_core = run_cpu_one_core(1.6, args.cpu_one_core_budget)

    import torch

    from paper_2405_05155_amd import inputs as I
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)

    if args.kappa:
        w = I.taylor_green_2d(nside=args.nside2d)
        one = run_gpu(w, args.kappa, args.steps2d, args.steps2d)
        print(json.dumps({"kappa": args.kappa, **one, "avg_launch_us": one["ms"] * 1e3 / one["launches"]}),
              flush=True)
        return
    if args.relax_iters:
        from paper_2405_05155_amd import sph as S
        from paper_2405_05155_amd import warmstart as WS
        ctx = S.Context(3)
        wr = I.sphere_fill(dx=1.0 / args.relax_nside, seed=2)
        run, _, _ = WS.relax_plain(ctx, wr, max_iter=args.relax_iters)
        print(json.dumps({"relax_iterations": run.iterations, "seconds": run.seconds, "residue": run.residue,
                          "n_particles": wr.n}), flush=True)
        return
    if args.setup:
        print(json.dumps(run_setup()), flush=True)
        return
    if args.plate:
        print(json.dumps({"kappa": args.plate, **run_plate(args.plate, args.steps_plate, 40)}), flush=True)
        return
    if args.shear:
        print(json.dumps(shear_layer_section()), flush=True)
        return
    if args.compressible:
        print(json.dumps(compressible_section()), flush=True)
        return
    if args.error_analysis:
        print(json.dumps(error_analysis_section()), flush=True)
        return
    if args.train_steps:
        print(json.dumps(run_train(args.train_steps)), flush=True)
        return
    if args.kappa3d:
        one = run_euler_3d(args.nside3d, args.kappa3d, args.steps, args.warmup)
        one.pop("_vel")
        print(json.dumps({"kappa": args.kappa3d, **one}), flush=True)
        return

    log(f"3-D Taylor-Green {args.nside3d}^3: {args.warmup} + {args.steps} Heun steps per cut-off")
    tw3 = run_euler_3d(args.nside3d, 1.6, args.steps, args.warmup, accuracy_steps=200)
    sw3 = run_euler_3d(args.nside3d, 2.0, args.steps, args.warmup, accuracy_steps=200)
    acc3 = tgv3d_accuracy(tw3, sw3, 0.01)
    tw3.pop("_vel"), sw3.pop("_vel")
    torch.cuda.empty_cache()

    from paper_2405_05155_amd.hbm_copy import copy_bandwidth
    copy_gbs = copy_bandwidth() / 1e9
    sha = source_sha(*STAGE_SOURCES)
    launch_s = tw3["avg_launch_us"] * 1e-6
    valu = None
    if VALU.get(sha, {}).get("3d"):
        insts = VALU[sha]["3d"]
        busy = insts * 4.0 / (VALU_SIMDS * VALU_CLOCK_HZ * launch_s)
        valu = {"insts_per_launch": insts, "issue_frac": busy,
                "note": "SQ_INSTS_VALU (wave instructions, counter profile) x 4 cycles / "
                        "(1,024 SIMDs x 2.4 GHz x launch time)"}
    out = {
        "metric": METRIC,
        "value": tw3["interactions_per_s"],
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": tw3["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"taylor_green_3d_{args.nside3d}^3_heun_kappa1.6", "n_particles": tw3["n_particles"],
                   "h_over_dx": 1.3, "c": 10.0, "nu": 0.01, "dt": tw3["dt"], "nnz_1.6h": tw3["nnz"],
                   "nnz_2h": sw3["nnz"]},
        "sw_2h": {"value": sw3["interactions_per_s"], "ms_per_step": sw3["ms_per_step"]},
        "speedup_tw_over_sw": sw3["ms_per_step"] / tw3["ms_per_step"],
        "accuracy": acc3,
        "roofline": {"bound": "hbm", "achieved": tw3["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": tw3["achieved_GBs"] / HBM_PEAK_GBS,
                     "traffic": TRAFFIC.get(sha, {}).get("3d"),
                     "kernel": "k_euler (3-D Heun stage, 1.6h)",
                     "avg_launch_us": tw3["avg_launch_us"], "bytes_per_launch": tw3["bytes_per_launch"],
                     "measured_copy_GBs": copy_gbs, "valu": valu},
        "taylor_green_3d": {"kappa1.6": tw3, "kappa2": sw3},
    }
    if not args.no_extra:
        log(f"2-D Taylor-Green {args.nside2d}^2: {args.steps2d} + {args.steps2d} Heun steps per cut-off")
        w2 = I.taylor_green_2d(nside=args.nside2d)
        tw, sw = run_gpu(w2, 1.6, args.steps2d, args.steps2d), run_gpu(w2, 2.0, args.steps2d, args.steps2d)
        launch2 = tw["ms"] * 1e-3 / tw["launches"]
        bytes2 = stage_bytes_2d(w2.n, tw["nnz"])
        out["taylor_green_2d"] = {
            "nside": args.nside2d, "steps_timed": args.steps2d, "steps_untimed_first": args.steps2d,
            "kappa1.6": {"interactions_per_s": tw["interactions_per_s"], "ms_per_step": tw["ms_per_step"],
                         "nnz": tw["nnz"]},
            "kappa2": {"interactions_per_s": sw["interactions_per_s"], "ms_per_step": sw["ms_per_step"],
                       "nnz": sw["nnz"]},
            "speedup_tw_over_sw": sw["ms_per_step"] / tw["ms_per_step"],
            "accuracy": {"t": 2 * args.steps2d * w2.meta["dt"], "vel_l2_err_tw": tw["vel_l2_err"],
                         "vel_l2_err_sw": sw["vel_l2_err"], "ratio_tw_over_sw": tw["vel_l2_err"] / sw["vel_l2_err"],
                         "reference": "decaying Taylor-Green velocity u0 exp(-8 pi^2 nu t)"},
            "roofline": {"bound": "hbm", "achieved": bytes2 / launch2 / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": bytes2 / launch2 / 1e9 / HBM_PEAK_GBS, "traffic": TRAFFIC.get(sha, {}).get("2d"),
                         "kernel": "k_euler (2-D Heun stage, 1.6h)", "avg_launch_us": launch2 * 1e6,
                         "bytes_per_launch": bytes2}}
        log("total-Lagrangian plate")
        twp, swp = run_plate(1.6, args.steps_plate, 40), run_plate(2.0, args.steps_plate, 40)
        out["tlsph_plate"] = {"kappa1.6": twp, "kappa2": swp,
                              "speedup_tw_over_sw": swp["ms_per_step"] / twp["ms_per_step"]}
        if args.plate_accuracy_steps:
            ht = plate_tip_history(1.6, args.plate_accuracy_steps, 100)
            hs = plate_tip_history(2.0, args.plate_accuracy_steps, 100)
            out["tlsph_plate"]["accuracy"] = {
                "steps": args.plate_accuracy_steps, "tip_deflection_sw_final": float(hs[-1]),
                "tip_deflection_tw_final": float(ht[-1]),
                "tip_history_diff_over_sw_amplitude": float(np.abs(ht - hs).max() / np.abs(hs).max())}
        log("double shear layer")
        out["double_shear_layer"] = shear_layer_section()
        log("compressible rows")
        out["compressible"] = compressible_section()
        log("error analysis")
        out["error_analysis"] = error_analysis_section()
    if not args.no_relax:
        log("relaxation: training and plain / warm-started runs")
        out["relax"] = run_relax(args.relax_epochs, args.relax_nside)
    if not args.no_cpu_baseline:
        log("oracle on the host cores: 3-D headline workload")
        torch.cuda.empty_cache()
        cpu = run_cpu_3d(args.cpu_budget, nside=args.nside3d)
        cpu["host"] = host_cpu()
        cpu["gpu_over_cpu"] = out["value"] / cpu["value"]
        if not args.no_extra:
            log("oracle on the host cores: plate, relaxation, 2-D workload")
            cpu["plate"] = run_cpu_plate(args.cpu_budget_extra)
            cpu["plate"]["gpu_over_cpu"] = out["tlsph_plate"]["kappa1.6"]["interactions_per_s"] / cpu["plate"]["value"]
            cpu["relax"] = run_cpu_relax(args.cpu_budget_extra, nside=args.relax_nside)
            cpu["taylor_green_2d"] = run_cpu_baseline(I.taylor_green_2d(nside=args.nside2d), 1.6,
                                                      args.cpu_budget_extra)
        if one_core is not None:
            cpu["one_core"] = one_core
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
