"""Benchmark of the AdResS hot path on one MI355X.

Workload (headline): 64,000 rigid-geometry tetrahedra (256,000 atoms) at molecular
density 0.1, x-slab atomistic region (half-width 10) + hybrid layer (5), atom WCA,
CG WCA (sigma 2.31) between centres of mass, harmonic bonds, FP32 pair arithmetic
with FP64 sums and FP64 velocity Verlet (dt 0.005), Verlet skin 0.3 rebuilt on
displacement.  Synthetic, seeded input (lattice + random orientations, Maxwell-
Boltzmann velocities at T = 1).

One "step" = one velocity-Verlet MD step through adres_integrate: kick-drift with
centres of mass and weights, list rebuild when needed (cells + Verlet), Eq. (1)
forces with the closing half-kick.  Prints one JSON line.

The second half of the metric, learned vs tabulated CG force, is measured on 256,000
CG sites (a centre frame of the headline geometry tiled 2 x 2 x 1, cutoff 3.0): frames
of centres and mapped forces from an all-atomistic Langevin run made by the library,
a force-matched cubic table (least squares, host) and the network trained on the GPU
on the same frames, held-out force RMSE of each (and of the plain method's CG force and of
the network's FP8 E4M3 variant), then MD steps/s of the 256k-site CG liquid with the table,
the network (BF16 matrix cores) and its FP8 variant.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "pair interactions/s + MD steps/s (AdResS 256k sites); learned vs tabulated CG"
EQUIL_SEED = 20181
EQUIL_GAMMA = 1.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--equilibrate", type=int, default=2000,
                    help="Langevin steps (gamma 1, kT 1, fixed seed) that melt the lattice start "
                         "before anything is timed; every timed run starts from that state")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cg-compare", action="store_true",
                    help="skip the learned-vs-tabulated CG force leg")
    ap.add_argument("--cg-steps", type=int, default=500)
    ap.add_argument("--cg-only", action="store_true",
                    help="run only the learned-vs-tabulated CG force leg and print its record")
    ap.add_argument("--no-hamiltonian", action="store_true",
                    help="skip the potential-energy-interpolation (Eq. (2)) leg")
    ap.add_argument("--no-tdforce", action="store_true",
                    help="skip the thermodynamic-force (correction field) leg")
    ap.add_argument("--no-respa", action="store_true",
                    help="skip the multiple-time-stepping (RESPA) leg")
    ap.add_argument("--no-anchors", action="store_true",
                    help="skip the self-adjusting (anchor spheres) region leg")
    ap.add_argument("--no-c5", action="store_true",
                    help="skip the 1M-tetrahedron heterogeneous run inside the learned-CG leg")
    ap.add_argument("--no-c1-c3", action="store_true",
                    help="skip the small FP64 workload (C1) and the Kremer-Grest melt (C3) legs")
    ap.add_argument("--workload", default="c2",
                    help="c2 (the headline) or c5 (1,000,000 tetrahedra, spherical AT region); "
                         "the CG force is the analytic WCA between centres")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device-to-device copy of this many bytes 10 times "
                         "(reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only (no multi-GPU path); --gpus must be 1"}))
        sys.exit(2)

    import torch

    if args.copy_bytes:
        src = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_bytes, "launches": 10}))
        return

    from paper_1806_10841_amd import inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.cg_only:
        print(json.dumps({"learned_vs_tabulated": learned_vs_tabulated(args.cg_steps, not args.no_c5)}))
        return
    wl = inputs.workload(args.workload)
    if wl.cg_kind != inputs.CG_WCA:
        # the force-matched table and the network are fitted inside the learned leg only
        wl = wl.with_(cg_kind=inputs.CG_WCA)
    x, v = inputs.make_state(wl)
    rec = timed_workload(wl, x, v, args.steps, args.warmup, args.equilibrate, gamma=0.0)

    out = {
        "metric": METRIC,
        "value": rec["steps_per_s"],
        "unit": "MD steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair arithmetic, f64 sums and integration",
        "data": "synthetic",
        "config": {
            "workload": f"{wl.name}: {wl.n_mol} tetrahedra ({wl.n_mol * wl.sites_per_mol} atoms), "
                        f"{'x-slab' if wl.region == inputs.REGION_SLAB_X else 'sphere'} AdResS "
                        f"AT {wl.d_at:g} + HY {wl.d_hy:g}, WCA atoms + WCA CG, harmonic bonds, "
                        f"NVE velocity Verlet dt {wl.dt:g}; timed from a melted state ({args.equilibrate} "
                        f"Langevin steps, gamma {EQUIL_GAMMA:g}, kT 1, from the lattice start)",
            "n_mol": wl.n_mol, "n_sites": wl.n_mol * wl.sites_per_mol, "box": wl.box[0],
            "list_rebuilds": rec["list_rebuilds"], "equilibration_steps": args.equilibrate,
        },
    }
    for k in ("pair_interactions_per_s", "interacting_pairs_per_eval", "listed_molecule_pairs",
              "listed_pairs_per_s", "force_kernel_us", "force_kernel_launches_timed",
              "steps_per_s_median_of_5", "steps_per_s_of_5"):
        out[k] = rec[k]
    traffic = _measured_traffic() if wl.name == "c2" else None   # counters were taken on C2
    avg_s = rec["force_kernel_us"] * 1e-6
    copy_gbs = _copy_bandwidth_gbs(torch)
    out["roofline"] = {
        "bound": "hbm",
        "achieved": rec["achieved_GBps"],
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": rec["achieved_GBps"] / HBM_PEAK_GBS,
        "traffic": traffic,
        "kernel": "k_forces<4,float,step> (Eq. 1 + bonds + closing kick, opening kick + drift)",
        "bytes_per_launch": rec["bytes_per_launch"],
        # counter bytes over the same time, against the peak (None without counters)
        "traffic_frac": None if traffic is None else traffic / avg_s / 1e9 / HBM_PEAK_GBS,
        # achievable HBM on this GPU: a plain 1 GiB device copy (read + write bytes)
        "copy_GBps": copy_gbs,
        "frac_of_copy": rec["achieved_GBps"] / copy_gbs,
    }
    valu = _measured_valu_insts() if wl.name == "c2" else None
    # the bound the kernel actually meets: its VALU instructions (counters) at the issue rate
    # of every SIMD, against the same launch time
    out["roofline"]["valu_issue"] = None if valu is None else {
        "wave_instructions_per_launch": valu, "peak_wave_instructions_per_s": VALU_WAVE_INSTS_PER_S,
        "issue_us": 1e6 * valu / VALU_WAVE_INSTS_PER_S, "frac": valu / VALU_WAVE_INSTS_PER_S / avg_s}
    x_eq, v_eq = rec.pop("_state")

    if not args.no_c1_c3 and wl.name == "c2":
        out["c1_fp64_small"] = c1_leg()
        out["c3_kremer_grest"] = c3_leg(args.steps, args.warmup)
    if not args.no_hamiltonian:
        out["hamiltonian_scheme"] = hamiltonian_leg(wl, x_eq, v_eq, args.steps, args.warmup)
    if not args.no_tdforce:
        out["thermodynamic_force"] = tdforce_leg(wl, x, v, args.steps)
    if not args.no_respa:
        out["respa"] = respa_leg(wl, x_eq, v_eq, args.steps, args.warmup, rec["steps_per_s"])
    if not args.no_anchors:
        out["self_adjusting_region"] = anchors_leg(wl, x, v, args.steps, args.warmup, args.equilibrate)
    if not args.no_cg_compare:
        out["learned_vs_tabulated"] = learned_vs_tabulated(args.cg_steps, not args.no_c5)

    if not args.no_cpu_baseline and wl.name == "c2":   # the oracle's all-pairs steps: C2 only
        out["cpu_baseline"] = cpu_baseline(wl, x_eq, v_eq)
    print(json.dumps(out))


def timed_workload(wl, x, v, steps, warmup, equilibrate, gamma=0.0, kT=1.0, seed=3, eq_gamma=EQUIL_GAMMA):
    """MD steps/s of adres_integrate on workload wl from a fixed melted state: equilibrate
    Langevin steps (fixed seed) from (x, v), then warmup untimed steps, then the timed call
    (and five repeats, and one with HIP events on every force launch) each restarted from the
    equilibrated state, so that the timed state depends on neither --steps nor --warmup.
    Also the fused step's average duration, its algorithmic bytes and rate, and the pair
    counts of the equilibrated state."""
    import torch
    from scipy.spatial import cKDTree
    from paper_1806_10841_amd import binding
    ctx = binding.Context(wl)
    xt = torch.tensor(x, device="cuda")
    vt = torch.tensor(v, device="cuda")
    ft = torch.empty_like(xt)
    if equilibrate:
        ctx.integrate(xt, vt, ft, wl.dt, equilibrate, gamma=eq_gamma, kT=1.0, seed=EQUIL_SEED)
    torch.cuda.synchronize()
    x_eq, v_eq = xt.clone(), vt.clone()
    ctx.integrate(xt, vt, ft, wl.dt, warmup, gamma=gamma, kT=kT, seed=seed)
    torch.cuda.synchronize()

    def run(evented):
        xt.copy_(x_eq)
        vt.copy_(v_eq)
        if evented:
            ctx.kernel_timing(True, every=1)       # events on every force launch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nreb = ctx.integrate(xt, vt, ft, wl.dt, steps, gamma=gamma, kT=kT, seed=seed)
        torch.cuda.synchronize()
        return steps / (time.perf_counter() - t0), nreb

    sps, nreb = run(False)
    # five repeats without events: their median rate (a spread check beside value), then
    # one with HIP events on every force launch for the kernel's duration (the events slow
    # the launch stream by a few per cent, so value and the median are taken without them)
    rates = [run(False)[0] for _ in range(5)]
    run(True)
    force_ms, launches = ctx.kernel_timing(False)
    avg_s = force_ms / 1e3 / max(launches, 1)

    # workload statistics of the equilibrated state (measurement only)
    xt.copy_(x_eq)
    n_pairs = ctx.build_verlet(xt)
    com, w = ctx.weights(xt)
    torch.cuda.synchronize()
    xf, comf, wf = xt.cpu().numpy(), com.cpu().numpy(), w.cpu().numpy()
    ctx.close()
    box = np.asarray(wl.box)
    spm = wl.sites_per_mol
    pts = np.mod(xf.T, box)
    mol = np.arange(xf.shape[1]) // spm
    ap_ = cKDTree(pts, boxsize=box).query_pairs(wl.rc_at, output_type="ndarray")
    ma, mb = mol[ap_[:, 0]], mol[ap_[:, 1]]
    n_at = int(np.count_nonzero((ma != mb) & (wf[ma] * wf[mb] > 0)))
    n_cg = 0
    if wl.region != inputs_region_all_at():
        cp = cKDTree(np.mod(comf.T, box), boxsize=box).query_pairs(wl.rc_cg, output_type="ndarray")
        n_cg = int(np.count_nonzero(wf[cp[:, 0]] * wf[cp[:, 1]] < 1))
    n_inter = n_at + n_cg
    # dominant kernel: the fused step launch (Eq. (1) forces at x_n, closing half-kick,
    # opening half-kick and drift to x_{n+1}), one per step.  Algorithmic bytes per launch:
    # positions read and written, velocities read and written (4 x 24 B per site), the
    # full neighbour list (4 B per entry, both directions of each listed pair) and the
    # row counts (4 B per molecule).  Derived per-molecule data and re-reads are the
    # implementation's, not the algorithm's, and are not counted; the measured HBM traffic
    # is reported beside it.
    ns, nm = wl.n_mol * spm, wl.n_mol
    bytes_per_launch = 96 * ns + 4 * 2 * n_pairs + 4 * nm
    return {
        "steps_per_s": sps, "ms_per_step": 1e3 / sps, "list_rebuilds": nreb,
        "steps_per_s_median_of_5": float(np.median(rates)), "steps_per_s_of_5": rates,
        "force_kernel_us": avg_s * 1e6, "force_kernel_launches_timed": launches,
        "pair_interactions_per_s": n_inter / avg_s,
        "interacting_pairs_per_eval": {"at_atom_pairs": n_at, "cg_com_pairs": n_cg},
        "listed_molecule_pairs": n_pairs, "listed_pairs_per_s": n_pairs / avg_s,
        "bytes_per_launch": bytes_per_launch, "achieved_GBps": bytes_per_launch / avg_s / 1e9,
        "_state": (x_eq.cpu().numpy(), v_eq.cpu().numpy()),
    }


def inputs_region_all_at():
    from paper_1806_10841_amd import inputs
    return inputs.REGION_ALL_AT


def c1_leg(steps=100, reps=5):
    """512 tetrahedra, FP64 pairs (latency-bound: about 0.1 MB per evaluation): microseconds
    per force evaluation (adres_forces, each call synchronised) and per velocity-Verlet step
    (100-step adres_integrate calls from the lattice start, median of five)."""
    import torch
    from paper_1806_10841_amd import binding, inputs
    wl = inputs.workload("c1")
    x, v = inputs.make_state(wl)
    ctx = binding.Context(wl)
    xt = torch.tensor(x, device="cuda")
    vt = torch.tensor(v, device="cuda")
    ft = torch.empty_like(xt)
    for _ in range(20):
        ctx.forces(xt, ft)
    torch.cuda.synchronize()
    n_eval = 200
    t0 = time.perf_counter()
    for _ in range(n_eval):
        ctx.forces(xt, ft)
        torch.cuda.synchronize()
    us_eval = (time.perf_counter() - t0) / n_eval * 1e6
    ctx.integrate(xt, vt, ft, wl.dt, steps)
    per = []
    for _ in range(reps):
        xt.copy_(torch.tensor(x, device="cuda"))
        vt.copy_(torch.tensor(v, device="cuda"))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.integrate(xt, vt, ft, wl.dt, steps)
        torch.cuda.synchronize()
        per.append((time.perf_counter() - t0) / steps * 1e6)
    ctx.close()
    return {"workload": "c1: 512 tetrahedra, x-slab AT 4 + HY 3, FP64 pairs, NVE velocity Verlet dt 0.005",
            "us_per_force_eval": us_eval, "us_per_step_median_of_5": float(np.median(per)),
            "us_per_step_of_5": per, "steps": steps}


def c3_leg(steps, warmup, equilibrate=500):
    """1000 Kremer-Grest chains of 200 beads (200,000 beads, density 0.85), FENE + WCA, the
    plain method (w = 1), Langevin gamma 0.5 kT 1 at dt 0.01, as the workload states; timed
    from a state equilibrated by the same thermostat."""
    from paper_1806_10841_amd import inputs
    wl = inputs.workload("c3")
    x, v = inputs.make_state(wl)
    rec = timed_workload(wl, x, v, steps, warmup, equilibrate, gamma=wl.gamma, kT=wl.kT, seed=5,
                         eq_gamma=wl.gamma)
    rec.pop("_state")
    rec["workload"] = (f"c3: {wl.n_mol} beads in chains of {wl.chain_len}, FENE k {wl.k_bond:g} R0 {wl.r0_bond:g} "
                       f"+ WCA, Langevin gamma {wl.gamma:g} kT {wl.kT:g}, dt {wl.dt:g}")
    rec["roofline"] = {"bound": "hbm", "achieved": rec["achieved_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": rec["achieved_GBps"] / HBM_PEAK_GBS,
                       "kernel": "k_forces<1,float,step> (WCA + FENE + closing kick, Langevin BAOAB)"}
    return rec


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(wl, x, v, n_vv=2, n_sample=2000):
    """The FP64 oracle as it stands (all-pairs Eq. (1) forces, no neighbour list), timed on
    this host on the equilibrated headline state: one full force evaluation and n_vv
    velocity-Verlet steps on all threads, and the forces of a sample of molecules on one
    thread (extrapolated to the whole evaluation)."""
    import oracle
    m = oracle.Model(wl)
    threads = oracle.num_threads()
    t = time.perf_counter()
    m.forces(x)
    t_force = time.perf_counter() - t
    t = time.perf_counter()
    m.vv(x, v, wl.dt, n_vv)           # n_vv + 1 full Eq. (1) evaluations and n_vv VV updates
    t_vv = time.perf_counter() - t
    sel = np.sort(np.random.default_rng(9).choice(wl.n_mol, n_sample, replace=False))
    oracle.set_num_threads(1)
    try:
        t = time.perf_counter()
        m.forces_sampled(x, sel)
        t_one = time.perf_counter() - t
    finally:
        oracle.set_num_threads(threads)
    return {
        "value": n_vv / t_vv,
        "unit": "MD steps/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{n_vv} oracle velocity-Verlet steps on the full {wl.n_mol}-molecule equilibrated state "
                  f"({n_vv + 1} all-pairs Eq. (1) force evaluations, {t_vv:.1f} s on {threads} threads); "
                  f"one more evaluation alone, and the forces of {n_sample} sampled molecules on 1 thread",
        "cpu_model": _cpu_model(),
        "host_cpus": os.cpu_count(),
        "force_eval_s_all_threads": t_force,
        "force_eval_s_one_thread_extrapolated": t_one * wl.n_mol / n_sample,
        "one_thread_sample": {"molecules": n_sample, "seconds": t_one},
    }


def hamiltonian_leg(wl, x, v, steps, warmup):
    """The same workload and step with potential energy interpolation (Eq. (2)): pair
    weights (w_a + w_b) / 2 and the drift force on hybrid molecules.  Reports MD steps/s,
    the fused step kernel's average duration and the total energy (kinetic + potential)
    before and after the timed steps (NVE: the scheme conserves it)."""
    import torch
    from paper_1806_10841_amd import binding, inputs
    wh = wl.with_(scheme=inputs.SCHEME_HAMILTONIAN)
    masses = np.tile(np.asarray(wh.site_mass, dtype=np.float64), wh.n_mol)
    ctx = binding.Context(wh)
    xt = torch.tensor(x, device="cuda")
    vt = torch.tensor(v, device="cuda")
    ft = torch.empty_like(xt)

    def total_energy():
        _, e = ctx.forces(xt, energy=True)
        vv = vt.cpu().numpy()
        return float(e.sum().item() + 0.5 * np.sum(masses * (vv * vv).sum(axis=0)))

    ctx.integrate(xt, vt, ft, wh.dt, warmup)
    e0 = total_energy()
    torch.cuda.synchronize()
    ctx.kernel_timing(True, every=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nreb = ctx.integrate(xt, vt, ft, wh.dt, steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    force_ms, launches = ctx.kernel_timing(False)
    e1 = total_energy()
    ctx.close()
    return {
        "steps_per_s": steps / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "force_kernel_us": force_ms / max(launches, 1) * 1e3,
        "list_rebuilds": nreb,
        "total_energy_start": e0,
        "total_energy_end": e1,
        "energy_drift_per_molecule": (e1 - e0) / wh.n_mol,
    }


def anchors_leg(wl, x, v, steps, warmup, equilibrate, counts=(16, 256)):
    """Self-adjusting AT region (Sec. 2.5) on the same molecules: the union of spheres
    (radius 5, hybrid shell 4) around k anchor molecules that move with the simulation,
    weights recomputed from the nearest anchor after every step, with the Langevin
    thermostat (gamma 1, kT 1) that force interpolation needs (Sec. 2.3: no conserved
    energy; molecules switched to atomistic inside moving spheres otherwise heat up).
    Started from the lattice (x, v) and melted with its own region for `equilibrate`
    steps: a state melted with another AT region holds overlapping atoms in what would
    become atomistic here.  MD steps/s per k."""
    import torch
    from paper_1806_10841_amd import binding, inputs
    out = {}
    for k in counts:
        wk = wl.with_(region=inputs.REGION_SPHERES, d_at=5.0, d_hy=4.0)
        ctx = binding.Context(wk)
        ctx.set_anchors(inputs.anchor_molecules(wk.n_mol, k, 5))
        xt = torch.tensor(x, device="cuda")
        vt = torch.tensor(v, device="cuda")
        ft = torch.empty_like(xt)
        ctx.integrate(xt, vt, ft, wk.dt, equilibrate + warmup, gamma=1.0, kT=1.0, seed=11)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nreb = ctx.integrate(xt, vt, ft, wk.dt, steps, gamma=1.0, kT=1.0, seed=12)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        _, w = ctx.weights(xt)
        wn = w.cpu().numpy()
        ctx.close()
        out[f"anchors_{k}"] = {"steps_per_s": steps / el, "list_rebuilds": nreb,
                               "equilibration_steps": equilibrate,
                               "fraction_at": float((wn == 1.0).mean()),
                               "fraction_hybrid": float(((wn > 0) & (wn < 1)).mean())}
    return out


def respa_leg(wl, x, v, steps, warmup, vv_steps_per_s):
    """Multiple time stepping (Sec. 2.6) on the same workload: the CG part of Eq. (1) on
    an outer step of n_inner inner steps (dt 0.005), the atomistic part and bonds on every
    inner step.  Reports inner MD steps/s for n_inner = 2 and 4 (the same simulated time
    per step as the headline) and the ratio to plain velocity Verlet, with the analytic CG
    force and with a learned CG force (a randomly initialised network of the library's
    architecture, scale 0.3, above r = 2.2 with the plain CG force's table below, evaluated
    on BF16 matrix cores; the network is the costly part that the outer step saves)."""
    import torch
    from paper_1806_10841_amd import binding, cgtrain, inputs
    out = {}
    for cg in ("wca", "mlp"):
        wk = wl if cg == "wca" else wl.with_(cg_kind=inputs.CG_MLP)
        base = vv_steps_per_s if cg == "wca" else None
        for n_inner in ((2, 4) if cg == "wca" else (1, 2, 4)):
            ctx = binding.Context(wk)
            if cg == "mlp":
                # the plain CG force as the table below r_min = 2.2 (the repulsive core), the
                # network from there to the cutoff
                ctx.set_cg_table(*cgtrain.wca_table())
                ctx.mlp_set(inputs.mlp_init(12).astype(np.float32), wk.rc_cg, 0.3, 0.3, 2.2)
            xt = torch.tensor(x, device="cuda")
            vt = torch.tensor(v, device="cuda")
            ft = torch.empty_like(xt)
            ctx.integrate_respa(xt, vt, ft, wk.dt, n_inner, max(warmup // n_inner, 1))
            torch.cuda.synchronize()
            n_outer = max(steps // n_inner, 1)
            t0 = time.perf_counter()
            nreb = ctx.integrate_respa(xt, vt, ft, wk.dt, n_inner, n_outer)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            ctx.close()
            sps = n_outer * n_inner / el
            if base is None:
                base = sps          # n_inner = 1 of the learned CG force is its VV
            out[f"{cg}_n_inner_{n_inner}"] = {"inner_steps_per_s": sps, "speedup_vs_vv": sps / base,
                                              "list_rebuilds": nreb}
    return out


def smooth_counts(counts, width, h):
    """A binned histogram smoothed with a Gaussian of the given width (bin width h; the
    weights renormalised where the kernel leaves the table), rounded back to whole counts
    for the library's update (half a count against ~1e5 per bin).  width 0: unchanged."""
    counts = np.asarray(counts, dtype=np.int64)
    if width <= 0:
        return counts
    k = np.arange(len(counts))
    W = np.exp(-0.5 * (((k[:, None] - k[None, :]) * h) / width) ** 2)
    W /= W.sum(axis=1, keepdims=True)
    return np.rint(W @ counts.astype(np.float64)).astype(np.int64)


def number_fluctuation_s0(frames, box, lo, width, sides=(5, 8, 11, 14, 20)):
    """Long-wavelength limit of the structure factor, S(0) = rho k_B T kappa_T, from the
    variance-to-mean ratio of molecule counts in cubes tiling a slab of the box: x in
    [lo, lo + width) (periodic in x too; lo measured from the box's low corner), all of y
    and z.  Cubes of side L_y / m for m in `sides` (those that fit at least once across the
    slab); the ratio S_l approaches S(0) as a / l for a cube of side l (its surface term),
    so S(0) is the intercept of a least-squares line in 1 / l.  frames: centres (3, n) per
    frame, any image.  Returns (S0, {l: S_l})."""
    Lx, Ly, Lz = box
    out = {}
    for m in sides:
        l = Ly / m
        nx = int(width // l)
        if nx < 1:
            continue
        cnts = []
        for com in frames:
            u = (com[0] - lo) % Lx
            ok = u < nx * l
            ix = np.floor(u[ok] / l).astype(np.int64)
            iy = np.floor((com[1][ok] % Ly) / l).astype(np.int64) % m
            mz = int(round(Lz / l))
            iz = np.floor((com[2][ok] % Lz) / (Lz / mz)).astype(np.int64) % mz
            cnts.append(np.bincount((ix * m + iy) * mz + iz, minlength=nx * m * mz))
        c = np.concatenate(cnts).astype(np.float64)
        out[l] = float(c.var() / c.mean())
    ls = np.array(sorted(out))
    A = np.stack([np.ones_like(ls), 1.0 / ls], axis=1)
    s0 = float(np.linalg.lstsq(A, np.array([out[l] for l in ls]), rcond=None)[0][0])
    return s0, out


# Refinement schedule of the thermodynamic force: (iterations, prefactor as a fraction of
# k_B T / (rho_0 S(0)), Gaussian smoothing width of the profile).  The full prefactor cancels
# the long-wavelength deviation in one step (linear response: an external potential change
# dU shifts the density by -rho_0 S(k) dU / k_B T at wavenumber k), but a dense liquid's S(k)
# grows far above S(0) toward its first peak, where that gain would diverge: the coarse phase
# takes half of it on a profile smoothed over 1.5 sigma, the next ones smaller fractions on
# finer profiles to remove the layering the coarse phase cannot see.
TD_SCHEDULE = ((6, 0.5, 1.5), (5, 0.1, 0.5), (8, 0.05, 0.0))


def tdforce_leg(wl, x, v, steps, n_bins=14, relax=4000, sample_steps=16000, sample_every=40,
                equilibrate=40000, s0_frames=100):
    """Thermodynamic force (Sec. 2.4) on the same workload: a correction table over the
    hybrid layer plus one sigma on each side, refined from density profiles of a Langevin
    run (gamma 1, kT 1) that first melts the lattice start for `equilibrate` steps.  The
    prefactor comes from the measured compressibility: S(0) from number fluctuations in the
    AT and the CG region (the larger, the more compressible phase, sets k_B T / (rho_0 S(0))),
    then the iterations of TD_SCHEDULE, each `relax` steps after the table change and then
    `sample_steps` sampled every `sample_every`.  Reports the largest deviation
    |rho / rho_0 - 1| over all bins and over the hybrid bins per iteration and of a final
    sample, the wall time per iteration, the density-profile kernel's cost, and MD steps/s
    of the plain step with the final correction installed."""
    import torch
    from paper_1806_10841_amd import binding
    lo, hi = wl.d_at - 1.0, wl.d_at + wl.d_hy + 1.0
    rho0 = wl.n_mol / float(np.prod(wl.box))
    ctx = binding.Context(wl)
    ctx.set_tdforce(np.zeros(n_bins), lo, hi)
    xt = torch.tensor(x, device="cuda")
    vt = torch.tensor(v, device="cuda")
    ft = torch.empty_like(xt)
    h = (hi - lo) / n_bins
    vol = 2.0 * h * wl.box[1] * wl.box[2]
    counts = torch.zeros(n_bins, dtype=torch.int64, device="cuda")
    centres = lo + (np.arange(n_bins) + 0.5) * h
    hy = (centres > wl.d_at) & (centres < wl.d_at + wl.d_hy)
    seed = 7
    ctx.integrate(xt, vt, ft, wl.dt, equilibrate, gamma=1.0, kT=1.0, seed=seed)   # melt the lattice
    # S(0) of the two phases from frames of the uncorrected run
    frames = []
    for k in range(s0_frames):
        seed += 1
        ctx.integrate(xt, vt, ft, wl.dt, 50, gamma=1.0, kT=1.0, seed=seed)
        com, _ = ctx.weights(xt)
        frames.append(com.cpu().numpy())
    c0 = wl.center[0]
    s0_at, sl_at = number_fluctuation_s0(frames, wl.box, c0 - (wl.d_at - 2.0), 2.0 * (wl.d_at - 2.0))
    cg_lo = c0 + wl.d_at + wl.d_hy + 2.0
    s0_cg, sl_cg = number_fluctuation_s0(frames, wl.box, cg_lo, wl.box[0] - 2.0 * (wl.d_at + wl.d_hy + 2.0))
    s0 = max(s0_at, s0_cg)
    p_full = 1.0 / (rho0 * s0)   # k_B T = 1

    def sample():
        nonlocal seed
        seed += 1
        ctx.integrate(xt, vt, ft, wl.dt, relax, gamma=1.0, kT=1.0, seed=seed)
        counts.zero_()
        nfr = sample_steps // sample_every
        for _ in range(nfr):
            seed += 1
            ctx.integrate(xt, vt, ft, wl.dt, sample_every, gamma=1.0, kT=1.0, seed=seed)
            tp = time.perf_counter()
            ctx.density_profile(xt, counts)
            torch.cuda.synchronize()
            prof[0] += time.perf_counter() - tp
            prof[1] += 1
        c = counts.cpu().numpy()
        dev = c / (nfr * vol) / rho0 - 1.0
        return c, nfr, dev

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prof = [0.0, 0]
    devs, devs_hy, iters = [], [], 0
    for n_it, frac, width in TD_SCHEDULE:
        for _ in range(n_it):
            c, nfr, dev = sample()
            devs.append(float(np.abs(dev).max()))
            devs_hy.append(float(np.abs(dev[hy]).max()))
            ctx.tdforce_update(torch.tensor(smooth_counts(c, width, h), device="cuda"), nfr, frac * p_full)
            iters += 1
    _, _, dev = sample()   # the profile with the final table
    torch.cuda.synchronize()
    cycle_s = (time.perf_counter() - t0) / (iters + 1)
    table = ctx.get_tdforce()
    # plain NVE steps with the final correction installed
    ctx.integrate(xt, vt, ft, wl.dt, 100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.integrate(xt, vt, ft, wl.dt, steps)
    torch.cuda.synchronize()
    sps = steps / (time.perf_counter() - t0)
    ctx.close()
    return {
        "bins": n_bins, "range": [lo, hi], "hybrid_bins": int(hy.sum()),
        "s0_at": s0_at, "s0_cg": s0_cg, "s0_by_cube_side_at": {f"{l:.3f}": s for l, s in sl_at.items()},
        "s0_by_cube_side_cg": {f"{l:.3f}": s for l, s in sl_cg.items()},
        "prefactor_full": p_full,
        "schedule": [{"iterations": n, "prefactor": f * p_full, "smoothing_sigma": w} for n, f, w in TD_SCHEDULE],
        "relax_steps": relax, "sample_steps": sample_steps, "sample_every": sample_every,
        "max_density_deviation_before": devs[0],
        "max_density_deviation_hybrid_bins_before": devs_hy[0],
        "max_density_deviation_after": float(np.abs(dev).max()),
        "max_density_deviation_hybrid_bins_after": float(np.abs(dev[hy]).max()),
        "density_deviation_after": [float(d) for d in dev],
        "max_density_deviation_per_iteration": devs,
        "max_density_deviation_hybrid_bins_per_iteration": devs_hy,
        "equilibration_steps": equilibrate,
        "seconds_per_iteration": cycle_s,
        "density_profile_call_us": 1e6 * prof[0] / max(prof[1], 1),
        "steps_per_s_with_correction": sps,
        "final_table": [float(t) for t in table],
    }


PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_forces_step_c2_pmc.md")
KERNEL_SOURCES = ("paper_1806_10841_amd/csrc/k_forces.hip", "paper_1806_10841_amd/csrc/adres_internal.h")


def kernel_source_digest():
    """SHA-256 over the force kernel's sources (identifies the kernel the counters saw)."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _copy_bandwidth_gbs(torch, nbytes=1 << 30, reps=10):
    """Achievable HBM bandwidth: the best of reps device-to-device copies of nbytes,
    counting the bytes read and written."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b) / 1e3)
    del src, dst
    return 2 * nbytes / best / 1e9


def _pmc_fields():
    """Fields of the committed rocprofv3 counter summary of the force kernel ("key: value"
    lines and "| counter | value |" rows), or None when there is none or the kernel's
    sources changed since the counters were taken."""
    try:
        with open(PMC_SUMMARY) as f:
            text = f.read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        line = line.strip()
        if line.startswith("|"):
            cells = [c.strip() for c in line.strip("|").split("|")]
            if len(cells) == 2:
                fields[cells[0]] = cells[1].replace(",", "")
            continue
        line = line.lstrip("-* ").strip()
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip().strip("`")] = v.strip().strip("`")
    if fields.get("source_sha256") != kernel_source_digest():
        return None
    return fields


def _measured_traffic():
    """HBM bytes per launch of the force kernel from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy's readings), or None."""
    fields = _pmc_fields()
    try:
        return float(fields["traffic_bytes_per_launch"]) if fields else None
    except (KeyError, ValueError):
        return None


# One wave64 VALU instruction issues every 4 cycles per SIMD (16 lanes; packed FP32 is not
# used, so FP32 and FP64 issue alike): 1,024 SIMDs x 2.4 GHz / 4.
VALU_WAVE_INSTS_PER_S = 1024 * 2.4e9 / 4


def _measured_valu_insts():
    """VALU wave instructions per launch of the force kernel (SQ_INSTS_VALU) from the
    committed counter summary, or None."""
    fields = _pmc_fields()
    try:
        return float(fields["SQ_INSTS_VALU"]) if fields else None
    except (KeyError, ValueError):
        return None


def learned_vs_tabulated(cg_steps, with_c5=True):
    """Force RMSE and MD steps/s of the learned and the tabulated CG force (256k sites)."""
    import torch
    from paper_1806_10841_amd import binding, cgtrain, inputs

    t_all = time.perf_counter()
    n_frames, n_train = 40, 32
    com, fmap, box = cgtrain.generate_frames(40, n_frames, stride=20, warmup=400, seed=7)
    tr, te = slice(0, n_train), slice(n_train, n_frames)
    com_np, fm_np = com.cpu().numpy(), fmap.cpu().numpy()
    r_min = cgtrain.min_pair_distance(com_np[:4], box, quantile=1e-4)
    table = cgtrain.fit_table(com_np[:8], fm_np[:8], box, r_fit_lo=r_min)
    params, scale, hist = cgtrain.train_mlp(com[tr], fmap[tr], box, steps=300, lr=2e-3, batch=4,
                                            r_min=r_min, table=table)
    tw = 0.5
    mlp = (params, scale, tw, r_min)
    rmse = {
        "plain_cg_wca": cgtrain.rmse_on_device(com[te], fmap[te], box, inputs.CG_WCA),
        "fm_table": cgtrain.rmse_on_device(com[te], fmap[te], box, inputs.CG_TABLE, table=table),
        "mlp": cgtrain.rmse_on_device(com[te], fmap[te], box, inputs.CG_MLP, table=table, mlp=mlp),
        "mlp_fp8": cgtrain.rmse_on_device(com[te], fmap[te], box, inputs.CG_MLP_FP8, table=table, mlp=mlp),
    }
    c4, box4 = cgtrain.tile_frame(com_np[-1], box, (2, 2, 1))
    n4 = c4.shape[1]
    v4 = inputs.maxwell_velocities(n4, np.full(n4, 4.0), 1.0, np.random.default_rng(1004))
    runs = {}
    for name, kind in (("table", inputs.CG_TABLE), ("mlp", inputs.CG_MLP), ("mlp_fp8", inputs.CG_MLP_FP8)):
        ctx = binding.Context(cgtrain.cg_workload(n4, box4, kind))
        ctx.set_cg_table(*table)
        if kind != inputs.CG_TABLE:
            ctx.mlp_set(params, 3.0, scale, tw, r_min)
        xt = torch.tensor(inputs.wrap_into_box(c4, box4), device="cuda")
        vt = torch.tensor(v4, device="cuda")
        ft = torch.empty_like(xt)
        ctx.integrate(xt, vt, ft, 0.005, 50)
        ctx.kernel_timing(1, every=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nreb = ctx.integrate(xt, vt, ft, 0.005, cg_steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        f_ms, f_n = ctx.kernel_timing(0 if kind == inputs.CG_TABLE else 2, every=1)
        rec = {"steps_per_s": cg_steps / el, "list_rebuilds": nreb, "force_kernel_us": 1e3 * f_ms / max(f_n, 1)}
        if kind != inputs.CG_TABLE:
            ctx.integrate(xt, vt, ft, 0.005, cg_steps)
            m_ms, m_n = ctx.kernel_timing(0)
            rec["mlp_prepass_us"] = 1e3 * m_ms / max(m_n, 1)
        rec["listed_pairs"] = ctx.build_verlet(xt)
        ctx.close()
        runs[name] = rec
    c5 = large_heterogeneous(table, params, scale, tw, r_min) if with_c5 else None
    pairs = runs["mlp"]["listed_pairs"]
    flop_per_pair = 2 * 64 * 64 + 2 * 64 + 2 * 64 + 2
    mlp_tflops = flop_per_pair * pairs / (runs["mlp"]["mlp_prepass_us"] * 1e-6) / 1e12
    return {
        "workload": f"c4: {n4} CG sites (mass 4), box {box4[0]:.3f} x {box4[1]:.3f} x {box4[2]:.3f}, "
                    "cutoff 3.0, NVE velocity Verlet dt 0.005",
        "steps": cg_steps,
        "mlp_steps_per_s": runs["mlp"]["steps_per_s"],
        "mlp_fp8_steps_per_s": runs["mlp_fp8"]["steps_per_s"],
        "table_steps_per_s": runs["table"]["steps_per_s"],
        "force_rmse_heldout": rmse,
        "mapped_force_rms": cgtrain.force_scale(fmap[te]),
        "training": {"frames": f"{n_frames} frames of 64,000 tetrahedra (all-atomistic Langevin, "
                               f"stride 20 steps), {n_train} train / {n_frames - n_train} held out",
                     "adam_steps": len(hist), "loss_first": hist[0], "loss_last": hist[-1],
                     "r_min_table_fallback": r_min},
        "runs": runs,
        "mlp_prepass": {"pairs": pairs, "flop_per_pair": flop_per_pair, "tflops": mlp_tflops,
                        "frac_of_bf16_mfma_peak": mlp_tflops / 2500.0},
        "c5_large_heterogeneous": c5,
        "seconds": time.perf_counter() - t_all,
    }


def large_heterogeneous(table, params, scale, tw, r_min, steps=200, warmup=20):
    """1,000,000 tetrahedra with a spherical AT region (radius 12, hybrid shell 5) in a
    CG bath, FP32 pairs, NVE velocity Verlet dt 0.005: MD steps/s with the force-matched
    table, the trained network (BF16 matrix cores) and its FP8 variant as F^CG of Eq. (1),
    all with the CG cutoff 3.0 the network was trained for."""
    import torch
    from paper_1806_10841_amd import binding, inputs
    wl = inputs.workload("c5").with_(rc_cg=3.0)
    x, v = inputs.make_state(wl)
    out = {"workload": f"c5: {wl.n_mol} tetrahedra ({wl.n_mol * 4} atoms), sphere AT 12 + HY 5, CG cutoff 3.0, "
                       "FP32 pairs, NVE velocity Verlet dt 0.005", "steps": steps}
    for name, kind in (("table", inputs.CG_TABLE), ("mlp", inputs.CG_MLP), ("mlp_fp8", inputs.CG_MLP_FP8)):
        ctx = binding.Context(wl.with_(cg_kind=kind))
        ctx.set_cg_table(*table)
        if kind != inputs.CG_TABLE:
            ctx.mlp_set(params, 3.0, scale, tw, r_min)
        xt = torch.tensor(x, device="cuda")
        vt = torch.tensor(v, device="cuda")
        ft = torch.empty_like(xt)
        ctx.integrate(xt, vt, ft, wl.dt, warmup)
        ctx.kernel_timing(1, every=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nreb = ctx.integrate(xt, vt, ft, wl.dt, steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        f_ms, f_n = ctx.kernel_timing(0)
        ctx.close()
        out[name] = {"steps_per_s": steps / el, "list_rebuilds": nreb,
                     "force_kernel_us": 1e3 * f_ms / max(f_n, 1)}
    return out


if __name__ == "__main__":
    main()
