"""Benchmark: LDG Jacobian-vector product throughput and Newton-GMRES time-to-1e-8.

Headline workload: 3D compressible Navier-Stokes, Taylor-Green vortex (Re 1600,
Mach 0.1, Pr 0.71) on a periodic 64^3 hex mesh of (0, 2 pi)^3, LDG p=3, five
conserved variables: N = 64^3 * 64 * 5 = 83,886,080 DOF, the largest of the
configurations and the only one whose vectors exceed the last-level cache.

Timed steps: K applications of the FP64 Jacobian-vector product J(u) v with
q(u) cached as inside GMRES (ldg_jvp_prepared: the gradient kernel for the
tangent of q + the tangent residual kernel), at the BDF2 wrapper of a CFL-10
step, inputs resident in HBM.  value = N * K / (timed seconds) in GDOF/s.  After
the timed region the same run reports the FP32 product, the unprepared product,
the residual, the 3D Poisson workload (32^3 perturbed hexes: JVPs in every
precision mode and Newton-GMRES time-to-1e-8 for the plain FP64 block-Jacobi
form and the mixed forms), the other workload shapes, implicit steps, and the
oracle on a bounded sample of elements on the host (1 core).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


OPERATOR_SOURCES = ("ldg_device.hpp", "ldg_physics.hpp", "ldg_operator_kernels.hpp", "ldg_operator_launch.hpp")


def kernel_sources_sha256(kind_source):
    """Hash of the sources that define one model kind's operator kernels (names and contents)."""
    h = hashlib.sha256()
    for name in OPERATOR_SOURCES + (kind_source,):
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_2205_07824_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(profile, kind_source):
    """HBM bytes per JVP launch from a committed TCC counter summary, or None when the kernels changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.split(":", 1)[0] in ("traffic_bytes_per_launch", "sources_sha256"):
                k, v = line.split(":", 1)
                kv[k] = v.strip()
    if kv.get("sources_sha256") != kernel_sources_sha256(kind_source) or "traffic_bytes_per_launch" not in kv:
        return None
    return int(kv["traffic_bytes_per_launch"])


def host_info():
    """Host cores and CPU model of the machine the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def build_workload(ldg, I, n=32, p=3):
    import torch
    box = I.box_mesh(3, n, perturb=0.05, seed=0)
    m = ldg.Mesh(box, p)
    xn, xq, xb, _ = m.points()
    _, _, f = I.mms_expsin3d(xq)
    ub, _, _ = I.mms_expsin3d(xb)
    tau = (p + 1) ** 2 * n
    md = ldg.Model(m, ldg.MODEL_POISSON, 1, [1.0, tau, 0.0], src=f.reshape(m.E, 1, m.nqv),
                   bdata=ub.reshape(m.nbf, 1, m.nqf), bc_kind=(0,))
    return box, m, md


def ns_workload(ldg, I, n=64, p=3):
    """3D compressible Navier-Stokes Taylor-Green vortex (Re 1600, Mach 0.1, Pr 0.71) on a periodic n^3 hex mesh
    of (0, 2 pi)^3, LDG p=3, BDF2 wrapper at dt = 10 h / max(|v| + c) (CFL 10); u = the initial state, v a seeded
    U(-1, 1) direction."""
    import torch
    L = 2 * np.pi
    box = I.box_mesh(3, n, lo=(0, 0, 0), hi=(L, L, L), periodic=(True,) * 3)
    m = ldg.Mesh(box, p)
    xn, _, _, _ = m.points()
    Ut = I.taylor_green(xn)                                   # [E][nn][5]
    del xn
    rho = Ut[..., 0]
    vel = np.sqrt((Ut[..., 1:4] ** 2).sum(-1)) / rho
    pr = 0.4 * (Ut[..., 4] - 0.5 * rho * vel ** 2)
    dt = 10.0 * (L / n) / float((vel + np.sqrt(1.4 * pr / rho)).max())
    md = ldg.Model(m, ldg.MODEL_NS, 5, [1.4, 1600.0, 0.71, (p + 1) ** 2 * n / L])
    u = torch.as_tensor(np.ascontiguousarray(Ut.transpose(0, 2, 1)).reshape(-1), device="cuda")
    del Ut
    v = torch.as_tensor(np.random.default_rng(2).uniform(-1, 1, md.N), device="cuda")
    return box, m, md, u, v, ldg.Time(a0=1.5 / dt), dt


def event_time(fn, reps):
    import torch
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def other_workloads(ldg, I, log):
    import torch
    res = {}
    # 2D Euler, p=4, periodic 256^2 on [0,20]^2, four isentropic vortices, BDF2 wrapper at dt = 0.05
    box = I.box_mesh(2, 256, lo=(0, 0), hi=(20, 20), periodic=(True, True))
    m = ldg.Mesh(box, 4)
    xn, _, _, _ = m.points()
    U = I.isentropic_vortices(xn, I.vortex_centres(4, 20.0, 5.0, 0)).transpose(0, 2, 1).reshape(-1)
    md = ldg.Model(m, ldg.MODEL_EULER, 4, [1.4])
    u = torch.as_tensor(U, device="cuda")
    v = torch.as_tensor(np.random.default_rng(2).uniform(-1, 1, md.N), device="cuda")
    t = ldg.Time(a0=1.5 / 0.05)
    Jv = md.empty()
    for nm, pr in (("fp64", ldg.FP64), ("fp32", ldg.FP32)):
        md.jvp(u, v, time=t, out=Jv, prec=pr)
        e = event_time(lambda: md.jvp(u, v, time=t, out=Jv, prec=pr), 20)
        res[f"euler2d_p4_256sq_jvp_{nm}_gdofs"] = round(md.N / e / 1e9, 3)
    res["euler2d_p4_256sq_dof"] = md.N
    # the same physics as a run-time compiled model (user source, hipRTC at model creation)
    from paper_2205_07824_amd import physics as UP
    t0 = time.perf_counter()
    mu_ = ldg.Model(m, ldg.MODEL_USER, 4, [1.4], physics_source=UP.EULER_2D, has_q=False)
    res["euler2d_p4_user_physics_compile_s"] = round(time.perf_counter() - t0, 2)
    for nm, pr in (("fp64", ldg.FP64), ("fp32", ldg.FP32)):
        mu_.jvp(u, v, time=t, out=Jv, prec=pr)
        e = event_time(lambda: mu_.jvp(u, v, time=t, out=Jv, prec=pr), 20)
        res[f"euler2d_p4_256sq_user_physics_jvp_{nm}_gdofs"] = round(md.N / e / 1e9, 3)
    log("euler", res)
    del md, mu_, m, u, v, Jv
    torch.cuda.empty_cache()
    # the Poisson workload scaled to 96^3 (N = 56.6M, vectors larger than the 256 MB last-level cache)
    box, m, md = build_workload(ldg, I, n=96)
    v = torch.as_tensor(np.random.default_rng(2).uniform(-1, 1, md.N), device="cuda")
    Jv = md.empty()
    for nm, pr in (("fp64", ldg.FP64), ("fp32", ldg.FP32)):
        md.jvp(None, v, out=Jv, prec=pr)
        e = event_time(lambda: md.jvp(None, v, out=Jv, prec=pr), 20)
        res[f"poisson3d_p3_96cube_jvp_{nm}_gdofs"] = round(md.N / e / 1e9, 3)
        res[f"poisson3d_p3_96cube_jvp_{nm}_us"] = round(e * 1e6, 1)
    res["poisson3d_p3_96cube_dof"] = md.N
    log("poisson 96^3", res)
    del md, m, v, Jv, box
    torch.cuda.empty_cache()
    return res


def mfma_p4(ldg, I, log, steps=20):
    """2D Poisson p=4 on 512^2 quads (N = 6,553,600): the BF16/FP16-MFMA JVP (dense element contractions on the
    matrix cores) against the FP64 JVP; dense MFMA flops per JVP = 4 d nn^2 E (two GEMMs)."""
    import torch
    box = I.box_mesh(2, 512)
    m = ldg.Mesh(box, 4)
    md = ldg.Model(m, ldg.MODEL_POISSON, 1, [1.0, 25.0 * 512, 0.0], bc_kind=(0,))
    v = torch.as_tensor(np.random.default_rng(2).uniform(-1, 1, md.N), device="cuda")
    ref = md.jvp(None, v).clone()
    Jv = md.empty()
    res = {"workload": "2D Poisson p=4, 512^2 quads", "dof": md.N}
    flops = 4.0 * 2 * m.nn * m.nn * m.E
    for nm, pr in (("fp64", ldg.FP64), ("bf16_mfma", ldg.BF16_MFMA), ("fp16_mfma", ldg.FP16_MFMA)):
        md.jvp(None, v, out=Jv, prec=pr)
        e = event_time(lambda: md.jvp(None, v, out=Jv, prec=pr), steps)
        res[f"jvp_{nm}_gdofs"] = round(md.N / e / 1e9, 3)
        res[f"jvp_{nm}_us"] = round(e * 1e6, 1)
        if pr != ldg.FP64:
            res[f"jvp_{nm}_rel_err_vs_fp64"] = float(((Jv - ref).norm() / ref.norm()).item())
            res[f"jvp_{nm}_dense_mfma_tflops"] = round(flops / e / 1e12, 3)
    log("mfma p=4", res)
    del md, m, v, ref, Jv
    torch.cuda.empty_cache()
    return res


def other_solves(ldg, I, log):
    """Newton-GMRES time-to-tolerance on the 2D Poisson p=2 8x8 workload (Newton 1 step, GMRES(30) + block-Jacobi
    to 1e-10)."""
    import torch
    res = {}
    box = I.box_mesh(2, 8)
    m = ldg.Mesh(box, 2, 5)
    xn, xq, xb, _ = m.points()
    _, _, f = I.mms_sin2d(xq)
    ub, _, _ = I.mms_sin2d(xb)
    md = ldg.Model(m, ldg.MODEL_POISSON, 1, [1.0, 9.0 * 8, 0.0], src=f.reshape(m.E, 1, m.nqv),
                   bdata=ub.reshape(m.nbf, 1, m.nqf), bc_kind=(0,))
    for rep in range(2):   # the first solve also allocates the solver workspace
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pc = ldg.BlockJacobi(md)
        u = torch.zeros(md.N, dtype=torch.float64, device="cuda")
        u, st, status = ldg.newton(md, u, rtol=1e-10, eta=1e-11, maxit=4, pc=pc, restart=30, lin_maxit=500,
                                   check=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    res["poisson2d_p2_8x8"] = {"time_to_1e-10_s": round(el, 5), "converged": status == ldg.LDG_OK,
                               "gmres_iters": st["gmres_iters"], "dof": md.N}
    log("poisson 8x8", res["poisson2d_p2_8x8"])
    return res


LEARNED_NET = os.path.join(ROOT, "paper_2205_07824_amd", "data", "convdiff2d_p3_128sq_linear_mlp.npz")


def learned_leg(ldg, I, log, held_out=4, restart=512):
    """2D convection-diffusion p=3 on 128^2 quads (N = 262,144), held-out seeds 100000...: FGMRES(restart) to
    1e-8 from x = 0 with FP64 block-Jacobi alone and with the learned linear form (the network shipped with the
    package, trained by learned.py on seeds 0.. of the same workload); each time includes building its
    preconditioner."""
    import torch
    from paper_2205_07824_amd import learned as LP
    if not os.path.exists(LEARNED_NET):
        log("learned leg skipped: no trained network at", LEARNED_NET)
        return None
    net, info = LP.load_network(LEARNED_NET)
    rows = []
    for i, sd in enumerate(range(100000, 100000 + held_out)):
        inst = LP.c5_instance(sd, n=128, p=3)
        if i == 0:   # the first solve of this basis size allocates the solver workspace: not timed
            bj = ldg.BlockJacobi(inst["model"])
            ldg.gmres(inst["model"], inst["b"], pc=bj, restart=restart, maxit=2, check=False)
            del bj
        r = LP.evaluate(inst, net, restart=restart, rtol=1e-8, maxit=20000)
        r["seed"], r["A"] = sd, round(inst["A"], 3)
        rows.append(r)
        log("learned", sd, {k: (v["iters"], v["ok"], v["seconds"]) for k, v in r.items() if isinstance(v, dict)})
        del inst
    torch.cuda.empty_cache()
    return {"workload": "2D convection-diffusion, LDG p=3, 128^2 quads, log-normal kappa, divergence-free b "
                        "(|b| <= A, A ~ LogUniform[1, 100]), f = 1", "dof": 128 * 128 * 16,
            "solver": f"FGMRES({restart}) from x = 0 to 1e-8, FP64", "held_out_seeds": [r["seed"] for r in rows],
            "network": {k: info.get(k) for k in ("instances", "samples", "epochs", "dims", "n", "p")},
            "rows": [{"seed": r["seed"], "A": r["A"],
                      "block_jacobi": {k: r["block_jacobi"][k] for k in ("iters", "ok", "seconds")},
                      "learned": {k: r["learned"][k] for k in ("iters", "ok", "seconds", "fell_back")}}
                     for r in rows],
            "summary": LP.summarize(rows)}


def implicit_steps(ldg, I, log, nsteps=5):
    """2D Euler, four isentropic vortices, 256^2 p=4 periodic: BDF1 then BDF2 steps at CFL 10, each solved by
    Newton-GMRES(50) + block-Jacobi rebuilt per Newton iterate, eta = 1e-3, ||G|| <= 1e-8 ||G0|| (a block-Jacobi
    kept from the first iterate of each step, bj_refresh = 2, stalled GMRES(50) on this workload)."""
    import torch
    from paper_2205_07824_amd import timestep as TS
    box = I.box_mesh(2, 256, lo=(0, 0), hi=(20, 20), periodic=(True, True))
    m = ldg.Mesh(box, 4)
    xn, _, _, _ = m.points()
    Ut = I.isentropic_vortices(xn, I.vortex_centres(4, 20.0, 5.0, 0)).transpose(0, 2, 1)
    dt = TS.euler_cfl_dt(Ut, 2, 20.0 / 256, 10.0)
    md = ldg.Model(m, ldg.MODEL_EULER, 4, [1.4])
    u0 = torch.as_tensor(np.ascontiguousarray(Ut).reshape(-1), device="cuda")
    res = {"workload": "2D Euler p=4, 256^2 periodic [0,20]^2, 4 isentropic vortices, BDF2 at CFL 10",
           "dof": md.N, "dt": dt, "steps": nsteps}
    for name, jp, bp, rf in (("fp64_jvp+fp64_bj", ldg.FP64, ldg.FP64, 1), ("fp32_jvp+fp32_bj", ldg.FP32, ldg.FP32, 1),
                             ("fp32_jvp+fp16_bj", ldg.FP32, ldg.FP16, 1)):
        _, stats = TS.bdf_steps(md, u0, dt, nsteps, restart=50, eta=1e-3, rtol=1e-8, jvp_prec=jp, bj_prec=bp,
                                bj_refresh=rf, log=log)
        later = stats[1:] if len(stats) > 1 else stats
        res[name] = {"seconds_per_step_2_to_%d" % nsteps: round(float(np.mean([r["seconds"] for r in later])), 4),
                     "all_converged": all(r["converged"] for r in stats) and len(stats) == nsteps,
                     "newton_iters": [r["newton_iters"] for r in stats],
                     "gmres_iters": [r["gmres_iters"] for r in stats],
                     "t_jvp_s": round(sum(r["t_jvp"] for r in later), 4),
                     "t_pc_s": round(sum(r["t_pc"] for r in later), 4),
                     "t_orth_s": round(sum(r["t_orth"] for r in later), 4)}
        log(name, res[name])
    # the paper's integrator family: three steps of the L-stable three-stage DIRK(3,3) (each stage a
    # Newton-GMRES solve like one BDF2 step), mixed-precision form
    name = "fp32_jvp+fp16_bj_dirk33"
    _, stats = TS.dirk_steps(md, u0, dt, 3, scheme="dirk33", restart=50, eta=1e-3, rtol=1e-8, jvp_prec=ldg.FP32,
                             bj_prec=ldg.FP16, bj_refresh=1, log=log)
    later = stats[1:]
    res[name] = {"seconds_per_step_2_to_3": round(float(np.mean([r["seconds"] for r in later])), 4),
                 "all_converged": all(r["converged"] for r in stats) and len(stats) == 3,
                 "newton_iters": [r["newton_iters"] for r in stats],
                 "gmres_iters": [r["gmres_iters"] for r in stats]}
    log(name, res[name])
    del md, m, u0
    torch.cuda.empty_cache()
    return res


def ns_implicit_steps(ldg, I, log, nsteps=2, cfl=1.0):
    """64^3 Navier-Stokes Taylor-Green vortex: a BDF1 step, then BDF2 steps, at acoustic CFL `cfl`
    (dt = cfl h / max(|v| + c)), each solved by Newton-GMRES(40) + per-variable block-Jacobi (64 x 64 blocks,
    rebuilt once per step) to ||G|| <= 1e-8 ||G_0||, eta = 1e-3.  Seconds per step over steps 2..nsteps, in
    the plain FP64 form, the mixed form (FP32 JVP, FP16 factors; FP64 residual and Krylov vectors) and the
    mixed form with FP32 state (the preconditioned vectors and the linearization point in FP32)."""
    import torch
    from paper_2205_07824_amd import timestep as TS
    _, m, md, u0, _, _, dt10 = ns_workload(ldg, I)
    dt = dt10 * cfl / 10.0
    res = {"workload": "3D Navier-Stokes Taylor-Green vortex, p=3, periodic 64^3, BDF2 at acoustic CFL %g" % cfl,
           "dof": md.N, "dt": dt, "steps": nsteps}
    # the last form keeps the blocks of the first BDF2 step for the next two steps (rebuild every 3 steps)
    for name, jp, bp, s32, ns, every in (("fp64_jvp+fp64_bj", ldg.FP64, ldg.FP64, False, nsteps, 1),
                                         ("fp32_jvp+fp16_bj", ldg.FP32, ldg.FP16, False, nsteps, 1),
                                         ("fp32_state+fp16_bj", ldg.FP32, ldg.FP16, True, nsteps, 1),
                                         ("fp32_state+fp16_bj_rebuilt_every_3_steps", ldg.FP32, ldg.FP16, True,
                                          nsteps + 2, 3)):
        torch.cuda.synchronize()
        _, stats = TS.bdf_steps(md, u0, dt, ns, restart=40, eta=1e-3, rtol=1e-8, jvp_prec=jp, bj_prec=bp,
                                per_variable=True, bj_refresh=2, lin_maxit=3000, log=log, state32=s32,
                                bj_every=every)
        later = stats[1:] if len(stats) > 1 else stats
        res[name] = {"seconds_per_step_2_to_%d" % ns: round(float(np.mean([r["seconds"] for r in later])), 4),
                     "seconds_per_step": [round(r["seconds"], 4) for r in stats],
                     "blocks_rebuilt": [r["blocks_rebuilt"] for r in stats],
                     "all_converged": all(r["converged"] for r in stats) and len(stats) == ns,
                     "newton_iters": [r["newton_iters"] for r in stats],
                     "gmres_iters": [r["gmres_iters"] for r in stats],
                     "t_jvp_s": round(sum(r["t_jvp"] for r in later), 4),
                     "t_pc_s": round(sum(r["t_pc"] for r in later), 4),
                     "t_orth_s": round(sum(r["t_orth"] for r in later), 4)}
        log(name, res[name])
        torch.cuda.empty_cache()
    del md, m, u0
    torch.cuda.empty_cache()
    return res


# Newton-GMRES forms on the Poisson workload: (JVP precision, block-Jacobi factor
# storage, Newton forcing eta)
NEWTON_FORMS = {"fp64_jvp+fp64_bj": ("FP64", "FP64", 1e-9), "fp64_jvp+fp32_bj": ("FP64", "FP32", 1e-9),
                "fp64_jvp+fp16_bj": ("FP64", "FP16", 1e-9), "fp32_jvp+fp32_bj": ("FP32", "FP32", 1e-4),
                "fp32_jvp+fp16_bj": ("FP32", "FP16", 1e-4), "fp32_jvp+bf16_bj": ("FP32", "BF16", 1e-4),
                "fp32_state+fp16_bj": ("FP32", "FP16", 1e-4)}


def newton_form(ldg, md, name, orth, log, restart=30):
    """Block-Jacobi build + Newton-GMRES(restart) from u = 0 to ||G|| <= 1e-8 ||G(0)||, timed end to end."""
    import torch
    jp, bp, eta = NEWTON_FORMS[name]
    jp, bp = getattr(ldg, jp), getattr(ldg, bp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pc = ldg.BlockJacobi(md, prec=bp)
    torch.cuda.synchronize()
    t_bj = time.perf_counter() - t0
    x = torch.zeros(md.N, dtype=torch.float64, device="cuda")
    x, st, status = ldg.newton(md, x, rtol=1e-8, eta=eta, maxit=8, pc=pc, restart=restart, lin_maxit=4000,
                               jvp_prec=jp, orth=orth, state32=name.startswith("fp32_state"), check=False)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    rec = {"time_to_1e-8_s": round(t_all, 4), "bj_build_s": round(t_bj, 4),
           "converged": status == ldg.LDG_OK, "newton_iters": st["iters"], "gmres_iters": st["gmres_iters"],
           "res_ratio": st["res_final"] / max(st["res0"], 1e-300),
           "t_jvp_s": round(st["t_jvp"], 4), "t_pc_s": round(st["t_pc"], 4), "t_orth_s": round(st["t_orth"], 4)}
    log(name, rec)
    return rec


def bickley_jet_steps(ldg, I, log, nsteps=3):
    """Shallow-water Bickley jet, the paper's second convection workload: 128^2 periodic quads of (-2 pi, 2 pi)^2,
    p=4, g = 1e4, physics compiled at run time (user source), DIRK(3,3) at CFL 10 from the initial state, each
    stage Newton-GMRES(50) + block-Jacobi rebuilt per Newton iterate to ||G|| <= max(1e-8 ||G_0||, 1e-10).  The
    nearly steady jet starts each stage with ||G_0|| ~ 3e-3, while the FP64 residual bottoms out near 4e-11 (the
    rounding of the g h^2 / 2 = 5e3 pressure flux), so a relative 1e-8 alone is unreachable.  JVP throughput and
    seconds per step (steps 2..nsteps) in the FP64 and the mixed form."""
    import torch
    from paper_2205_07824_amd import timestep as TS
    from paper_2205_07824_amd import physics as UP
    L, n, g = 4.0 * np.pi, 128, 1.0e4
    box = I.box_mesh(2, n, lo=(-L / 2, -L / 2), hi=(L / 2, L / 2), periodic=(True, True))
    m = ldg.Mesh(box, 4)
    xn, _, _, _ = m.points()
    Ut = I.bickley_jet(xn, seed=0, eps=0.01)              # [E][nn][3]
    speed = np.sqrt(Ut[..., 1] ** 2 + Ut[..., 2] ** 2) / Ut[..., 0] + np.sqrt(g * Ut[..., 0])
    dt = 10.0 * (L / n) / float(speed.max())
    t0 = time.perf_counter()
    md = ldg.Model(m, ldg.MODEL_USER, 3, [g], physics_source=UP.SHALLOW_WATER_2D, has_q=False)
    res = {"workload": "shallow-water Bickley jet, p=4, 128^2 periodic quads of (-2pi, 2pi)^2, g = 1e4, "
                       "run-time compiled physics, DIRK(3,3) at CFL 10",
           "dof": md.N, "dt": dt, "physics_compile_s": round(time.perf_counter() - t0, 2)}
    u0 = torch.as_tensor(np.ascontiguousarray(Ut.transpose(0, 2, 1)).reshape(-1), device="cuda")
    v = torch.as_tensor(np.random.default_rng(2).uniform(-1, 1, md.N), device="cuda")
    t = ldg.Time(a0=1.0 / dt)
    Jv = md.empty()
    for nm, pr in (("fp64", ldg.FP64), ("fp32", ldg.FP32)):
        md.jvp(u0, v, time=t, out=Jv, prec=pr)
        e = event_time(lambda: md.jvp(u0, v, time=t, out=Jv, prec=pr), 20)
        res[f"jvp_{nm}_gdofs"] = round(md.N / e / 1e9, 3)
    for name, jp, bp in (("fp64_jvp+fp64_bj", ldg.FP64, ldg.FP64), ("fp32_jvp+fp16_bj", ldg.FP32, ldg.FP16)):
        _, stats = TS.dirk_steps(md, u0, dt, nsteps, scheme="dirk33", restart=50, eta=1e-3, rtol=1e-8, atol=1e-10,
                                 jvp_prec=jp, bj_prec=bp, bj_refresh=1, log=log)
        later = stats[1:] if len(stats) > 1 else stats
        res[name] = {"seconds_per_step_2_to_%d" % nsteps: round(float(np.mean([r["seconds"] for r in later])), 4),
                     "all_converged": all(r["converged"] for r in stats) and len(stats) == nsteps,
                     "newton_iters": [r["newton_iters"] for r in stats],
                     "gmres_iters": [r["gmres_iters"] for r in stats]}
        log(name, res[name])
    del md, m, u0, v, Jv
    torch.cuda.empty_cache()
    return res


def wave_displacement_steps(ldg, I, log, nsteps=4):
    """The paper's wave model with its displacement ODE (Eq. 1c, w_t = u, plus a nonlinear second component
    mu1 q1 q2): the plane wave w = sin(k.x - |k| t), k = 2 pi (2, 1), c = 1, on 256^2 periodic quads of the unit
    square, p=4, physics and ODE compiled at run time, DIRK(3,3) at CFL 5 (c dt / h), Newton-GMRES(50) +
    block-Jacobi to 1e-10.  JVP throughput, the ODE stage kernel's time and bandwidth (56 B per node: u, r1, w),
    seconds per step, and the displacement's error against the closed form."""
    import torch
    from paper_2205_07824_amd import timestep as TS
    from paper_2205_07824_amd import physics as UP
    n, p = 256, 4
    m = ldg.Mesh(I.box_mesh(2, n, periodic=(True, True)), p)
    xn, _, _, _ = m.points()
    k = 2 * np.pi * np.array([2.0, 1.0])
    om = float(np.linalg.norm(k))
    th = xn @ k                                            # [E][nn]
    U0 = np.stack([-om * np.cos(th), -k[0] * np.cos(th), -k[1] * np.cos(th)], axis=1).reshape(-1)
    dt = 5.0 / n
    t0 = time.perf_counter()
    md = ldg.Model(m, ldg.MODEL_USER, 3, [1.0, 0.5], physics_source=UP.WAVE_2D_W, has_q=False)
    res = {"workload": "wave model + displacement ODE, p=4, 256^2 periodic quads, plane wave k = 2pi(2,1), "
                       "DIRK(3,3) at CFL 5", "dof": md.N, "ode_components": md.nw, "dt": dt,
           "physics_compile_s": round(time.perf_counter() - t0, 2)}
    u0 = torch.as_tensor(U0, device="cuda")
    v = torch.as_tensor(np.random.default_rng(3).uniform(-1, 1, md.N), device="cuda")
    t = ldg.Time(a0=1.0 / dt)
    Jv = md.empty()
    for nm, pr in (("fp64", ldg.FP64), ("fp32", ldg.FP32)):
        md.jvp(u0, v, time=t, out=Jv, prec=pr)
        e = event_time(lambda: md.jvp(u0, v, time=t, out=Jv, prec=pr), 20)
        res[f"jvp_{nm}_gdofs"] = round(md.N / e / 1e9, 3)
    nodes = m.E * m.nn
    w0 = np.stack([np.sin(th), np.zeros_like(th)], axis=1).reshape(-1)
    wr = torch.as_tensor(w0, device="cuda")
    wo = torch.empty_like(wr)
    tw = ldg.Time(a0=1.0 / dt, r1=wr, c1=1.0 / dt)
    md.ode_stage(u0, tw, 1.0, 0.0, out=wo)
    e = event_time(lambda: md.ode_stage(u0, tw, 1.0, 0.0, out=wo), 50)
    res["ode_stage_us"] = round(e * 1e6, 2)
    # 92 MB of state, timed on the same buffers: the rate is the last-level cache's, not HBM's
    res["ode_stage_cache_gbs"] = round(56.0 * nodes / e / 1e9, 1)
    ode = TS.Ode(w=torch.as_tensor(w0, device="cuda"), alpha=1.0, beta=0.0)
    _, stats = TS.dirk_steps(md, u0.clone(), dt, nsteps, scheme="dirk33", restart=50, eta=1e-3, rtol=1e-10,
                             atol=1e-10, jvp_prec=ldg.FP64, bj_prec=ldg.FP64, bj_refresh=2, log=log, ode=ode)
    torch.cuda.synchronize()
    later = stats[1:] if len(stats) > 1 else stats
    w = ode.w.cpu().numpy().reshape(m.E, 2, m.nn)[:, 0]
    res["dirk33_fp64"] = {"seconds_per_step_2_to_%d" % nsteps: round(float(np.mean([r["seconds"] for r in later])), 4),
                          "all_converged": all(r["converged"] for r in stats) and len(stats) == nsteps,
                          "newton_iters": [r["newton_iters"] for r in stats],
                          "gmres_iters": [r["gmres_iters"] for r in stats]}
    res["displacement_max_error"] = float(np.abs(w - np.sin(th - om * nsteps * dt)).max())
    log("wave + ode", res)
    del md, m, u0, v, Jv, wr, wo, ode
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=32, help="elements per direction of the 3D Poisson workload")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--orth", choices=("dcgs2", "cgs2"), default="dcgs2",
                    help="Gram-Schmidt variant of the Newton-GMRES legs")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra-workloads", action="store_true",
                    help="skip the 2D Euler and 96^3 Poisson JVP throughput legs")
    ap.add_argument("--no-implicit", action="store_true",
                    help="skip the implicit time steps (Navier-Stokes, Euler, shallow water, wave)")
    ap.add_argument("--profile-jvp-only", action="store_true",
                    help="only the timed headline JVP steps (for counter collection)")
    ap.add_argument("--profile-poisson-only", action="store_true",
                    help="only the FP64 JVP of the 3D Poisson workload (for counter collection)")
    ap.add_argument("--profile-mfma-only", action="store_true",
                    help="only the 2D Poisson p=4 MFMA JVP leg (for counter collection)")
    ap.add_argument("--profile-solve-only", choices=sorted(NEWTON_FORMS), default=None,
                    help="only one Newton-GMRES form on the Poisson workload (for a kernel trace)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 512 MiB buffer 10 times (scales the HBM byte counters)")
    ap.add_argument("--profile-ns-only", action="store_true",
                    help="only --steps FP64 Jacobian-vector products of the 64^3 Navier-Stokes workload with q(u) "
                         "cached (for a kernel trace or counters)")
    ap.add_argument("--profile-bj-only", action="store_true",
                    help="only one per-variable block-Jacobi build (FP16 factors) of the 64^3 Navier-Stokes workload "
                         "at its linearization point (for a kernel trace)")
    ap.add_argument("--profile-wave-only", action="store_true",
                    help="only the wave model + displacement ODE leg (for a kernel trace)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1"}))
        sys.exit(2)

    import torch
    from paper_2205_07824_amd import inputs as I
    from paper_2205_07824_amd import ldg

    assert torch.cuda.is_available()
    if args.copy_calibration:
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        c = torch.empty_like(a)
        for _ in range(10):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_dispatch": a.numel() * 8, "copy_bytes_written_per_dispatch": a.numel() * 8}))
        return
    if args.profile_mfma_only:
        print(json.dumps(mfma_p4(ldg, I, log, steps=args.steps)))
        return
    if args.profile_wave_only:
        print(json.dumps(wave_displacement_steps(ldg, I, log)))
        return
    if args.profile_bj_only:
        _, m, md, u, v, t, _ = ns_workload(ldg, I)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pc = ldg.BlockJacobi(md, u_lin=u, time=t, per_variable=True, prec=ldg.FP16)
        torch.cuda.synchronize()
        print(json.dumps({"ns3d_tgv_p3_64cube_bj_build_fp16_s": round(time.perf_counter() - t0, 4)}))
        del pc
        return
    if args.profile_ns_only:
        _, m, md, u, v, t, _ = ns_workload(ldg, I)
        Jv = md.empty()
        res = {"dof": md.N}
        for name, pr in (("fp64", ldg.FP64), ("fp32", ldg.FP32)):
            md.jvp_prepare(u, pr)
            md.jvp_prepared(u, v, time=t, out=Jv, prec=pr)
            e = event_time(lambda: md.jvp_prepared(u, v, time=t, out=Jv, prec=pr), args.steps)
            log(f"ns 64^3 prepared JVP {name}: {e * 1e3:.3f} ms")
            res[f"ns3d_tgv_p3_64cube_prepared_jvp_{name}_ms"] = round(e * 1e3, 4)
        print(json.dumps(res))
        return
    if args.profile_solve_only:
        _, _, md = build_workload(ldg, I, n=args.n)
        orth = ldg.ORTH_DCGS2 if args.orth == "dcgs2" else ldg.ORTH_CGS2
        print(json.dumps(newton_form(ldg, md, args.profile_solve_only, orth, log)))
        return
    if args.profile_poisson_only:
        _, m, md = build_workload(ldg, I, n=args.n)
        v = torch.as_tensor(np.random.default_rng(2).uniform(-1, 1, md.N), device="cuda")
        Jv = md.empty()
        for _ in range(args.warmup):
            md.jvp(None, v, out=Jv)
        e = event_time(lambda: md.jvp(None, v, out=Jv), args.steps)
        print(json.dumps({"poisson3d_p3_jvp_fp64_us": round(e * 1e6, 2), "n": args.n}))
        return

    # ---- headline: FP64 J(u) v of the 64^3 Navier-Stokes workload, q(u) cached
    box_ns, m, md, u, v, t, dt = ns_workload(ldg, I)
    N = md.N
    log(f"workload: 64^3 Navier-Stokes TGV, E={m.E} nn={m.nn} N={N} colours={m.ncolors} dt={dt:.4g}")
    md.jvp_prepare(u, ldg.FP64)
    Jv = md.empty()

    def step():
        md.jvp_prepared(u, v, time=t, out=Jv, prec=ldg.FP64)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e_jvp = event_time(step, args.steps)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    value = N * args.steps / T / 1e9
    log(f"FP64 JVP (q cached): {e_jvp * 1e3:.3f} ms/launch (events), wall {T / args.steps * 1e3:.3f} ms/step")

    # roofline of the product: algorithmic bytes = read u and v, write Jv (24 B/DOF; the uniform mesh needs no
    # stored geometry)
    alg_bytes = 24.0 * N
    achieved = alg_bytes / e_jvp / 1e9
    out = {
        "metric": "LDG JVP GDOF/s + Newton-GMRES time-to-1e-8, plain FP64 vs mixed/learned",
        "value": round(value, 4),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(T / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D compressible Navier-Stokes Taylor-Green vortex (Re 1600, Mach 0.1, Pr 0.71), "
                               "LDG p=3 on a periodic 64^3 hex mesh of (0, 2pi)^3; FP64 J(u)v with q(u) cached, "
                               "BDF2 wrapper at CFL 10",
                   "dof": N, "elements": m.E, "p": 3, "variables": 5, "quadrature": "collocated Gauss-Legendre 4^3"},
        "roofline": {"bound": "hbm", "kernel": "ldg_jvp_prepared (k_grad: tangent of q; k_resid: tangent residual; "
                                               "FP64)",
                     "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": recorded_traffic("jvp_ns3d_tgv_p3_64cube_hbm_counters.md", "ldg_op_ns.hip"),
                     "alg_bytes_per_launch": alg_bytes, "launch_us": round(e_jvp * 1e6, 3)},
    }
    if args.profile_jvp_only:
        print(json.dumps(out))
        return

    # measured HBM copy bandwidth on this GPU in the same run (512 MiB device-to-device copy, read + write
    # bytes per second), reported beside the 8 TB/s datasheet peak the roofline fraction uses
    a_ = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
    c_ = torch.empty_like(a_)
    c_.copy_(a_)
    e_copy = event_time(lambda: c_.copy_(a_), 20)
    copy_gbs = 2.0 * a_.numel() * 8 / e_copy / 1e9
    out["roofline"]["measured_copy_gbs"] = round(copy_gbs, 1)
    out["roofline"]["frac_of_measured_copy"] = round(achieved / copy_gbs, 4)
    # the same product counting the read of the q(u) cache (3 x 8 B/DOF more)
    out["roofline"]["achieved_with_q_cache_read"] = round(48.0 * N / e_jvp / 1e9, 2)
    del a_, c_
    torch.cuda.empty_cache()

    extra = {"ns3d_tgv_p3_64cube_jvp_fp64_ms": round(e_jvp * 1e3, 4)}
    md.jvp_prepare(u, ldg.FP32)
    e32 = event_time(lambda: md.jvp_prepared(u, v, time=t, out=Jv, prec=ldg.FP32), 10)
    extra["ns3d_tgv_p3_64cube_jvp_fp32_ms"] = round(e32 * 1e3, 4)
    extra["ns3d_tgv_p3_64cube_jvp_fp32_gdofs"] = round(N / e32 / 1e9, 3)
    Jref = md.jvp_prepared(u, v, time=t, prec=ldg.FP64).clone()
    J32 = md.jvp_prepared(u, v, time=t, prec=ldg.FP32)
    extra["ns3d_tgv_p3_64cube_jvp_fp32_rel_err_vs_fp64"] = float(((J32 - Jref).norm() / Jref.norm()).item())
    del J32
    eu = event_time(lambda: md.jvp(u, v, time=t, out=Jv, prec=ldg.FP64), 5)
    extra["ns3d_tgv_p3_64cube_jvp_fp64_with_q_ms"] = round(eu * 1e3, 4)
    G = md.empty()
    er = event_time(lambda: md.residual(u, time=t, out=G), 5)
    extra["ns3d_tgv_p3_64cube_residual_fp64_ms"] = round(er * 1e3, 4)
    del G
    log("ns extra:", extra)

    # oracle on a bounded sample of elements, host, one core
    if not args.no_cpu:
        out["cpu_baseline"] = ns_cpu_baseline(box_ns, md, u, v, t, Jref, log)
    del md, m, u, v, Jv, Jref
    torch.cuda.empty_cache()

    # ---- the 3D Poisson workload (32^3 perturbed hexes): every precision mode, Newton-GMRES forms
    out["poisson3d_p3_32cube"] = poisson_legs(ldg, I, args, log)

    # JVP throughput on the other workload shapes (FP64 and FP32, HIP events)
    if not args.no_extra_workloads:
        out["other_workloads"] = other_workloads(ldg, I, log)
        out["mfma_p4"] = mfma_p4(ldg, I, log)

    if not args.no_solve:
        out["other_solves"] = other_solves(ldg, I, log)
        out["learned"] = learned_leg(ldg, I, log)

    # implicit time steps: the 64^3 Navier-Stokes workload, then the 2D Euler workload (seconds per step
    # averaged over steps 2..5)
    if not args.no_implicit:
        out["ns3d_tgv_implicit_steps"] = ns_implicit_steps(ldg, I, log)
        out["implicit_steps"] = implicit_steps(ldg, I, log)
        out["bickley_jet"] = bickley_jet_steps(ldg, I, log)
        out["wave_displacement"] = wave_displacement_steps(ldg, I, log)
    out["extra"] = extra
    print(json.dumps(out))


def ns_cpu_baseline(box, md, u, v, t, Jgpu, log, budget_s=15.0):
    """The oracle's FP64 J(u) v of the Navier-Stokes workload on a bounded sample of elements (each with the
    neighbourhood its q needs), on one host core, and the GPU product compared on the same rows."""
    try:
        import oracle as O
        om = O.Mesh(box, 3)
        omd = O.Model(O.MODEL_NS, 5, [float(x) for x in md._mu], a0=t.a0)
        uu, vv = u.cpu().numpy(), v.cpu().numpy()
        probe = np.arange(0, om.E, om.E // 64, dtype=np.int64)[:64]
        # each call has a fixed cost that does not depend on the sample size: two probe sizes separate it
        # from the cost per element, so that the sample fills the time budget
        om.sample(omd, uu, vv, probe[:8])
        t0 = time.process_time()
        om.sample(omd, uu, vv, probe[:8])
        t8 = time.process_time() - t0
        t0 = time.process_time()
        om.sample(omd, uu, vv, probe)
        t64 = time.process_time() - t0
        per = max((t64 - t8) / 56, 1e-9)
        fixed = max(t8 - 8 * per, 0.0)
        count = int(min(om.E, max(64, (budget_s - fixed) / per)))
        sel = np.unique(np.linspace(0, om.E - 1, count).astype(np.int64))
        t0 = time.process_time()
        _, Jv_s = om.sample(omd, uu, vv, sel)
        tc = time.process_time() - t0
        Jg = Jgpu.cpu().numpy().reshape(om.E, -1)[sel]
        err = float(np.linalg.norm(Jg - Jv_s) / np.linalg.norm(Jv_s))
        dofs = len(sel) * om.nn * 5
        res = {"value": round(dofs / tc / 1e9, 7), "unit": "GDOF/s", "cores": 1, "kind": "oracle",
               "sample": f"FP64 oracle J(u)v with q(u) formed on each element's neighbourhood, {len(sel)} of "
                         f"{om.E} elements of the 64^3 Navier-Stokes workload, {tc:.1f} s process time",
               "gpu_vs_oracle_rel_err_on_sample": err}
        res.update(host_info())
        log("cpu baseline", res)
        return res
    except Exception as ex:  # the oracle is optional on the measuring box
        log("cpu baseline skipped:", ex)
        return None


def poisson_legs(ldg, I, args, log):
    """3D Poisson p=3 on 32^3 perturbed hexes: the FP64 JVP (events), every other precision mode with its error,
    the residual, and Newton-GMRES time-to-1e-8 in the six forms."""
    import torch
    box, m, md = build_workload(ldg, I, n=args.n)
    N = md.N
    v = torch.as_tensor(np.random.default_rng(2).uniform(-1, 1, N), device="cuda")
    u = torch.as_tensor(np.random.default_rng(1).uniform(-1, 1, N), device="cuda")
    Jv = md.empty()
    for _ in range(5):
        md.jvp(None, v, out=Jv)
    e64 = event_time(lambda: md.jvp(None, v, out=Jv), 100)
    res = {"workload": f"3D Poisson LDG p=3, {args.n}^3 hexes, interior vertices perturbed +-5% h", "dof": N,
           "jvp_fp64_us": round(e64 * 1e6, 2), "jvp_fp64_gdofs": round(N / e64 / 1e9, 3)}
    alg = 16.0 * N + 192.0 * m.E
    res["jvp_fp64_roofline"] = {"alg_bytes": alg, "achieved_gbs": round(alg / e64 / 1e9, 1),
                                "frac": round(alg / e64 / 1e9 / HBM_PEAK_GBS, 4),
                                "traffic": recorded_traffic("jvp_poisson3d_p3_32cube_hbm_counters.md",
                                                            "ldg_op_poisson.hip")}
    Jref = md.jvp(None, v).clone()
    for nm, pr in (("fp32", ldg.FP32), ("bf16_mfma", ldg.BF16_MFMA), ("fp16_mfma", ldg.FP16_MFMA)):
        try:
            eb = event_time(lambda: md.jvp(None, v, out=Jv, prec=pr), 50)
            res[f"jvp_{nm}_gdofs"] = round(N / eb / 1e9, 3)
            res[f"jvp_{nm}_rel_err_vs_fp64"] = float(((Jv - Jref).norm() / Jref.norm()).item())
        except ldg.LDGError as ex:
            res[f"jvp_{nm}_gdofs"] = None
            log(nm, "jvp:", ex)
    G = md.empty()
    er = event_time(lambda: md.residual(u, out=G), 50)
    res["residual_fp64_gdofs"] = round(N / er / 1e9, 3)
    log("poisson:", res)
    if not args.no_solve:
        orth = ldg.ORTH_DCGS2 if args.orth == "dcgs2" else ldg.ORTH_CGS2
        res["newton_gmres"] = {name: newton_form(ldg, md, name, orth, log) for name in NEWTON_FORMS}
    del md, m, u, v, Jv, Jref, G
    torch.cuda.empty_cache()
    return res


if __name__ == "__main__":
    main()
