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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device-to-device copy of this many bytes 10 times "
                         "(reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from scipy.spatial import cKDTree

    if args.copy_bytes:
        src = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_bytes, "launches": 10}))
        return

    from paper_1806_10841_amd import binding, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    wl = inputs.workload(args.workload)
    x, v = inputs.make_state(wl)
    ctx = binding.Context(wl)
    xt = torch.tensor(x, device=dev)
    vt = torch.tensor(v, device=dev)
    ft = torch.empty_like(xt)

    ctx.integrate(xt, vt, ft, wl.dt, args.warmup)
    torch.cuda.synchronize()

    ctx.kernel_timing(True)            # start recording force-kernel events
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nreb = ctx.integrate(xt, vt, ft, wl.dt, args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    force_ms, launches = ctx.kernel_timing(False)
    elapsed = t1 - t0
    steps_per_s = args.steps / elapsed

    # workload statistics on the final state (measurement only)
    n_pairs = ctx.build_verlet(xt)
    com, w = ctx.weights(xt)
    torch.cuda.synchronize()
    xf, comf, wf = xt.cpu().numpy(), com.cpu().numpy(), w.cpu().numpy()
    box = np.asarray(wl.box)
    spm = wl.sites_per_mol
    pts = np.mod(xf.T, box)
    mol = np.arange(xf.shape[1]) // spm
    ap_ = cKDTree(pts, boxsize=box).query_pairs(wl.rc_at, output_type="ndarray")
    ma, mb = mol[ap_[:, 0]], mol[ap_[:, 1]]
    n_at = int(np.count_nonzero((ma != mb) & (wf[ma] * wf[mb] > 0)))
    cp = cKDTree(np.mod(comf.T, box), boxsize=box).query_pairs(wl.rc_cg, output_type="ndarray")
    n_cg = int(np.count_nonzero(wf[cp[:, 0]] * wf[cp[:, 1]] < 1))
    n_inter = n_at + n_cg

    # dominant kernel: Eq. (1) forces + closing half-kick, one launch per step (plus one
    # per rebuild and one initial evaluation)
    avg_force_s = force_ms / 1e3 / max(launches, 1)
    ns, nm = wl.n_mol * spm, wl.n_mol
    list_entries = 2 * n_pairs
    bytes_per_launch = (24 * ns            # x read
                        + 24 * ns          # F write
                        + 48 * ns          # v read + write (half-kick)
                        + 40 * nm          # centre (24), weight (8), rho (8) read
                        + 4 * list_entries + 4 * nm)   # neighbour list + row counts
    achieved = bytes_per_launch / avg_force_s / 1e9
    pair_rate = n_inter / avg_force_s

    out = {
        "metric": METRIC,
        "value": steps_per_s,
        "unit": "MD steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair arithmetic, f64 sums and integration",
        "data": "synthetic",
        "config": {
            "workload": f"{wl.name}: {wl.n_mol} tetrahedra ({ns} atoms), x-slab AdResS AT 10 + HY 5, "
                        "WCA atoms + WCA CG, harmonic bonds, NVE velocity Verlet dt 0.005",
            "n_mol": wl.n_mol, "n_sites": ns, "box": wl.box[0], "r_list": None,
            "list_rebuilds": nreb,
        },
        "pair_interactions_per_s": pair_rate,
        "interacting_pairs_per_eval": {"at_atom_pairs": n_at, "cg_com_pairs": n_cg},
        "listed_molecule_pairs": n_pairs,
        "force_kernel_us": avg_force_s * 1e6,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": "k_forces<4,float> (Eq. 1 + bonds + half-kick)",
            "bytes_per_launch": bytes_per_launch,
        },
    }

    if not args.no_cpu_baseline:
        import oracle
        m = oracle.Model(wl)
        t = time.perf_counter()
        m.vv(x, v, wl.dt, 1)          # two full Eq. (1) evaluations + one VV update
        dt_cpu = time.perf_counter() - t
        out["cpu_baseline"] = {
            "value": 1.0 / (dt_cpu / 2.0),
            "unit": "MD steps/s",
            "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "one oracle velocity-Verlet step on the full 64,000-molecule state "
                      "(two all-pairs Eq. (1) force evaluations); steps/s = 2 / elapsed",
        }
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
