#!/usr/bin/env python3
"""Throughput of the HMC hot path on one MI355X: site-trials/s of full sweeps (2 or 8
colour passes with an elastic zone solve for every real trial flip, the global stress
refresh every R sweeps and the texture histograms of the workload) on the large
workload: 128^3 periodic lattice, 26 neighbours / 8 colours, 4000 Voronoi grains with
Haar-random orientations, biaxial 150/150 MPa, kT = 0.7, 5^3 zone with 200 relaxation
steps, refresh every 10 sweeps (200 steps), 10-degree texture histograms on x and y every
10 sweeps.

Prints ONE JSON line on stdout (progress goes to stderr).  A step is one sweep.

Other workloads (--workload): batched (the 64-replica ensemble against the same replicas run
alone), adjoint (64^3 forward + backward of the stored energy), potts and refresh (the colour
pass and the explicit step on lattices beyond the caches, default 512^3), growth (the ten
60^3 zero-load grain-growth runs of Sec. 6 as one fused batch), texture (Sec. 7's ten 100^3
runs: coarsening, then 75 sub-loads to 30 MPa, each a quasi-static refresh and one sweep).
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

METRIC = "site-trials/sec incl. elastic zone solve (128^3, 5^3 zone) vs oracle; % roofline"
PEAK_FP32_TFLOPS = 157.3     # MI355X vector FP32 (256 CU x 2.4 GHz x 256 FLOP/clk)
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def zone_flops_per_solve(h: int, nr: int) -> float:
    """FP32 work of one zone solve as the method's per-unit figure: n_r [(2h+1)^3 200 +
    (2h+2)^3 12] FLOP (200 per voxel and relaxation step for strain, stress and corner
    forces, 12 per node for the heavy-ball update)."""
    nv, nn = (2 * h + 1) ** 3, (2 * h + 2) ** 3
    return nr * (200.0 * nv + 12.0 * nn)


def zone_flops_minimal(h: int, nr: int) -> float:
    """The least FP32 work of one zone solve in the separable form the kernels use: per
    relaxation step and voxel, the strain from the 8 corners (9 gradient entries as
    separable sums/differences: 24 + 3 shear sums), the 6x6 stress (36 FMA = 72) and the
    corner forces (transposed sums: 27); per node the heavy-ball update (3 x 4)."""
    nv, nn = (2 * h + 1) ** 3, (2 * h + 2) ** 3
    return nr * (126.0 * nv + 12.0 * nn)


REFRESH_BYTES_PER_NODE_STEP = 50.0   # read u, w (24 B) + write u, w (24 B) + spin (2 B)


def source_hash(*sources):
    """First 16 hex digits of the SHA-256 of a kernel's sources and the code-generation options
    the build gives them: counters taken on one build stay valid while both are unchanged."""
    import hashlib

    from paper_1009_0457_amd.build import SOURCE_FLAGS

    data = b""
    for source in sources:
        data += open(os.path.join(ROOT, "paper_1009_0457_amd", "csrc", source), "rb").read()
        flags = SOURCE_FLAGS.get(source, [])
        if flags:
            data += ("\n// build: " + " ".join(flags)).encode()
    return hashlib.sha256(data).hexdigest()[:16]


# the lane-shift zone solve of the 5^3 zone: its template and the unit that instantiates it
ZONE_H2_SOURCES = ("hmc_zone_h2.hip", "hmc_zone_kernels.h")


def measured_traffic(key_bytes, key_hash, sources, summary="counters_large128.md"):
    """A figure (HBM bytes, executed operations) from a committed rocprofv3 counter summary,
    valid only while the kernel source still has the hash it had when the counters were taken
    (else None)."""
    try:
        vals = {}
        for line in open(os.path.join(ROOT, "profiles", summary)):
            if "=" in line and not line.startswith(("|", "`", "cd ")):
                k, v = (t.strip() for t in line.split("=", 1))
                vals[k] = v
        if source_hash(*((sources,) if isinstance(sources, str) else sources)) != vals.get(key_hash):
            return None
        return float(vals[key_bytes])
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--proposal", choices=["neighbor", "uniform"], default="neighbor",
                    help="neighbor: spin of a random neighbour slot (workload default); uniform: any other "
                         "state, which makes every trial a real flip (zone-solve saturation)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--saturation-steps", type=int, default=4,
                    help="large: sweeps of the uniform-proposal (every trial a zone solve) saturation line; 0 = off")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--K", type=int, default=0, help="override the lattice edge (diagnostics only)")
    ap.add_argument("--workload", choices=["large", "batched", "adjoint", "potts", "refresh", "growth", "texture"], default="large",
                    help="large: the headline 128^3 workload; batched: the 64-replica ensemble in fused "
                         "graph-captured launches vs the same replicas run one by one; adjoint: 64^3 "
                         "forward 2000 steps + backward with checkpoints every 50; potts: zero-load colour "
                         "passes on a lattice larger than the caches (default 512^3); refresh: explicit global "
                         "steps on such a lattice; growth: ten 60^3 zero-load grain-growth runs as one batch; "
                         "texture: the ten 100^3 runs of the loaded texture experiment as one batch")
    ap.add_argument("--neighbors", type=int, choices=[6, 26], default=None,
                    help="growth: 6 neighbours / 2 colours or 26 / 8 (default 26)")
    ap.add_argument("--zone-h", type=int, default=None, choices=[0, 1, 2, 3],
                    help="large: zone half-width other than the workload's 2 (a different configuration; "
                         "for the zone-size comparison)")
    ap.add_argument("--zone-steps", type=int, default=None, help="large: zone relaxation steps n_r")
    ap.add_argument("--material-points", type=int, choices=[1, 8], default=1,
                    help="refresh, texture: one material point per voxel (default) or 2x2x2 per cell of 2^3 sites")
    ap.add_argument("--replicas", type=int, default=64)
    ap.add_argument("--zone-variant", type=int, default=0, help="zone-solve kernel (0 = automatic)")
    ap.add_argument("--tile-z", type=int, default=0, help="node layers per block of the explicit step (0 = automatic)")
    ap.add_argument("--autotune", action="store_true",
                    help="batched: pick the explicit-step tile depth and the zone kernel with the autotuner "
                         "(tile depth on throw-away batches; zone kernel during the warm-up sweeps)")
    ap.add_argument("--zero-load", action="store_true",
                    help="the same lattice with no load: the elastic term is off and every trial is decided "
                         "by the integer threshold table inside the colour pass")
    ap.add_argument("--bandwidth-K", type=int, default=512,
                    help="large: also time the colour pass and the explicit step on the grain structure refined "
                         "to this edge (a multiple of 128; 0 skips)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (calibrates HBM byte counters)")
    return ap.parse_args()


def cpu_model():
    """The host CPU's model name (first 'model name' line of /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(lat, p, micro, seconds):
    """The FP64 oracle on a bounded sample of the same workload: random site-trials of one
    colour pass from the GPU's current state, plus one explicit step of the global solve;
    combined into site-trials/s of whole sweeps (K^3 trials plus refresh_steps/refresh_every
    explicit steps per sweep).  Serial (one thread: `value`), and as an aggregate of P threads
    each running the serial oracle on a disjoint part of the same pass's sites (P = the host's
    hardware threads, at most 16)."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    import oracle as O

    K = p.K
    lat.synchronize()
    spins = lat.get_spins().cpu().numpy()
    sig = lat.get_stress().cpu().numpy().astype(np.float64)
    s = lat.sweep_index()
    Ct, St, _ = O.tables(micro.euler, p.C11, p.C12, p.C44)
    prm = O.make_params(K, p.neighbors, micro.Q, proposal=p.proposal, h=p.zone_h, nr=p.zone_steps, elastic=True,
                        J=p.J, kT=p.kT, lambda_el=p.lambda_el, zone_alpha=p.zone_alpha, zone_beta=p.zone_beta,
                        seed=p.seed)
    rng = np.random.default_rng(123)
    # colour-0 sites: all coordinates even (8 colours) or x+y+z even (2 colours)
    g = np.arange(K)
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    mask = ((x & 1) == 0) & ((y & 1) == 0) & ((z & 1) == 0) if p.neighbors == 26 else ((x + y + z) & 1) == 0
    sites = np.nonzero(mask.ravel())[0]
    rng.shuffle(sites)
    done = 0
    t_trials = 0.0
    batch = 64
    while t_trials < seconds and done < sites.size:
        pick = sites[done:done + batch]
        t0 = time.perf_counter()
        O.trials(prm, spins, Ct, St, sig, s, pick)
        t_trials += time.perf_counter() - t0
        done += pick.size
        batch = min(4096, batch * 2)
    u = lat.get_displacement().cpu().numpy().astype(np.float64)
    E = lat.macro_strain()
    t0 = time.perf_counter()
    O.global_solve(K, spins, Ct, St, np.zeros(6), 1, False, p.glob_alpha, p.glob_beta, p.glob_alphaE, u=u, E=E)
    t_step = time.perf_counter() - t0
    t_sweep = K ** 3 * (t_trials / done) + (p.refresh_steps / p.refresh_every) * t_step
    # P threads: each a serial oracle call on its own chunk of further sites of the same pass
    # (the library call releases the interpreter lock); trials per chunk sized from the serial
    # rate so that the wall time is about seconds / 3
    P = max(1, min(16, os.cpu_count() or 1))
    per = max(8, int(done / t_trials * seconds / 3))
    rest = sites[done:]
    chunks = [rest[i * per:(i + 1) * per] for i in range(P) if i * per < rest.size]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(len(chunks)) as ex:
        list(ex.map(lambda c: O.trials(prm, spins, Ct, St, sig, s, c), chunks))
    t_par = time.perf_counter() - t0
    n_par = int(sum(c.size for c in chunks))
    t_sweep_par = K ** 3 * (t_par / n_par) + (p.refresh_steps / p.refresh_every) * t_step / len(chunks)
    return {
        "value": K ** 3 / t_sweep,
        "unit": "site-trials/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{done} random site-trials of colour pass 0 at sweep {s} from the GPU state "
                   f"({t_trials:.1f} s) + 1 explicit global step at {K}^3 ({t_step:.1f} s), combined as "
                   f"K^3 trials + {p.refresh_steps}/{p.refresh_every} steps per sweep; serial FP64 C, -O2"),
        "cpu_model": cpu_model(),
        "host_threads": os.cpu_count(),
        "aggregate": {"value": K ** 3 / t_sweep_par, "cores": len(chunks),
                      "sample": f"{n_par} further site-trials of the same pass in {len(chunks)} threads, one serial "
                                f"oracle call per thread on a disjoint chunk ({t_par:.1f} s wall); the explicit "
                                f"step taken as the serial one divided by the threads"},
    }


def small_configs():
    """The two small workloads end to end, on the GPU and in the serial oracle: the 16^3 tiny
    workload (6 neighbours, 8 grains, 100 MPa along z, 3^3 zone x 50 steps, a cold refresh and
    then a warm 200-step refresh before every one of its 10 sweeps) and the 64^3 workload's
    zero-load twin (26 neighbours, 500 grains, 100 sweeps; spins must agree bit for bit)."""
    import numpy as np
    import torch

    import oracle as O
    from paper_1009_0457_amd import hmc as H
    from paper_1009_0457_amd.synth import full_config, tiny_config

    out = {}
    for c in (tiny_config(), full_config().zero_load()):
        m = c.microstructure()
        elastic = bool(np.any(c.sigma_MPa != 0))
        p = H.hmc_default_params(c.K, c.neighbors, c.zone_h)
        p.kT, p.refresh_every, p.zone_steps, p.seed = c.kT, c.refresh_every, c.zone_steps, c.philox_seed
        if not elastic:
            p.lambda_el = 0.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat = H.Lattice(p, m.Q)
        lat.set_orientations(m.euler)
        lat.set_spins(m.spins)
        lat.set_load(c.sigma_MPa)
        if elastic:
            lat.stress_refresh(-1, True)
        lat.sweep(c.sweeps)
        gpu_spins = lat.get_spins().cpu().numpy()
        t_gpu = time.perf_counter() - t0
        lat.close()
        Ct, St, _ = O.tables(m.euler, p.C11, p.C12, p.C44)
        prm = O.make_params(c.K, c.neighbors, m.Q, proposal=p.proposal, h=p.zone_h, nr=p.zone_steps, elastic=elastic,
                            R=p.refresh_every, n_warm=p.refresh_steps, J=p.J, kT=p.kT, lambda_el=p.lambda_el,
                            zone_alpha=p.zone_alpha, zone_beta=p.zone_beta, glob_alpha=p.glob_alpha,
                            glob_beta=p.glob_beta, glob_alphaE=p.glob_alphaE, Sigma=np.asarray(c.sigma_MPa) * 1e-3,
                            seed=p.seed)
        q = m.spins.copy()
        t0 = time.perf_counter()
        if elastic:
            u, E, sig, _ = O.global_solve(c.K, q, Ct, St, np.asarray(c.sigma_MPa) * 1e-3, p.cold_steps, True,
                                          p.glob_alpha, p.glob_beta, p.glob_alphaE)
            u, E, sig = u.ravel().copy(), E.copy(), sig.ravel().copy()
        else:
            u = E = sig = np.zeros(1)
            E = np.zeros(6)
        O.sweeps(prm, q, Ct.ravel() if elastic else np.zeros(36 * m.Q), St.ravel() if elastic else np.zeros(36 * m.Q),
                 u, E, sig, 0, c.sweeps)
        t_ora = time.perf_counter() - t0
        n = c.sweeps * c.K ** 3
        out[c.name] = {"site_trials": n, "gpu_s": t_gpu, "oracle_s": t_ora,
                       "gpu_site_trials_per_s": n / t_gpu, "oracle_site_trials_per_s": n / t_ora,
                       "spins_equal": bool(np.array_equal(gpu_spins, q)),
                       "note": ("cold refresh + sweeps with a warm refresh before each, wall clock including the "
                                "library's set-up" if elastic else "zero load: integer decisions, spins bit-exact")}
        log(f"[bench] {c.name}: gpu {t_gpu:.3f} s, oracle {t_ora:.2f} s, spins equal {out[c.name]['spins_equal']}")
    return out


def bench_batched(a):
    """The replica ensemble: every replica of the batch in each launch, sweeps replayed from
    HIP graphs, against the same replicas run one after another as single lattices."""
    import numpy as np
    import torch

    from paper_1009_0457_amd import hmc as H
    from paper_1009_0457_amd.synth import batched_configs

    cfgs = batched_configs(a.replicas)
    log(f"[bench] building {len(cfgs)} replica microstructures")
    micros = []
    for i, c in enumerate(cfgs):
        micros.append(c.microstructure())
        if i % 16 == 15:
            log(f"[bench]   {i + 1} replicas built")
    common = H.hmc_default_params(16, 26, 2)
    common.refresh_every = cfgs[0].refresh_every
    common.refresh_tile_z = a.tile_z
    reps = []
    for c, m in zip(cfgs, micros):
        r = H.hmc_default_replica(common, c.K, m.Q)
        r.kT, r.seed = c.kT, c.philox_seed
        for i in range(6):
            r.sigma_MPa[i] = float(c.sigma_MPa[i])
        reps.append(r)
    sites = sum(c.K ** 3 for c in cfgs)
    tuned = None
    if a.autotune:
        from paper_1009_0457_amd import autotune as T

        def build(tz):
            q = H.hmc_params.from_buffer_copy(common)
            q.refresh_tile_z = tz
            bb = H.Batch(q, reps)
            for i, m in enumerate(micros):
                bb.set_replica(i, m.euler, m.spins)
            return bb

        tiles = T.tune_tile_depth(build)
        common.refresh_tile_z = tiles["best"]
        tuned = {"tile_z": tiles}
        log(f"[bench] autotune tile depth: {tiles}")
    b = H.Batch(common, reps)
    for i, m in enumerate(micros):
        b.set_replica(i, m.euler, m.spins)
    log(f"[bench] {sites} sites; cold refresh")
    b.stress_refresh(-1, True)
    if a.autotune:
        tuned["zone_variant"] = T.tune_zone_variant(b, common.zone_h)
        log(f"[bench] autotune zone kernel: {tuned['zone_variant']}")
    b.set_graphs(True)
    for _ in range(a.warmup):
        b.sweep(1)
    b.synchronize()
    b.reset_stats()
    t0 = time.perf_counter()
    b.sweep(a.steps)
    b.synchronize()
    t_batch = time.perf_counter() - t0
    st = b.stats()
    b.set_zone_screen(True)
    b.reset_stats()
    t0 = time.perf_counter()
    b.sweep(a.steps)
    b.synchronize()
    t_scr = time.perf_counter() - t0
    st_scr = b.stats()
    b_variant = tuned["zone_variant"]["best"] if tuned else common.zone_variant
    b.close()
    log(f"[bench] batch {t_batch:.3f} s ({sites * a.steps / t_batch:.4e} site-trials/s), screened {t_scr:.3f} s")
    # the same replicas one after another, each a single lattice with graph-replayed sweeps
    # (cold refresh and warm-up untimed)
    t_plain = 0.0
    for c, m, r in zip(cfgs, micros, reps):
        p = H.hmc_params.from_buffer_copy(common)
        p.refresh_tile_z = 0           # each lattice alone picks its own tile depth
        p.zone_variant = b_variant
        p.K, p.kT, p.lambda_el, p.seed = r.K, r.kT, r.lambda_el, r.seed
        p.glob_alpha, p.glob_beta, p.glob_alphaE = r.glob_alpha, r.glob_beta, r.glob_alphaE
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            lat = H.Lattice(p, m.Q, stream=s)
            lat.set_orientations(m.euler)
            lat.set_spins(m.spins)
            lat.set_load(list(r.sigma_MPa))
            lat.stress_refresh(-1, True)
            lat.set_graphs(True)
            for _ in range(a.warmup):
                lat.sweep(1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lat.sweep(a.steps)
            s.synchronize()
            t_plain += time.perf_counter() - t0
            lat.close()
    log(f"[bench] replicas alone: {t_plain:.3f} s")
    trials = sites * a.steps
    out = {
        "metric": "site-trials/sec of the replica ensemble (fused launches, graph-replayed sweeps)",
        "value": trials / t_batch, "unit": "site-trials/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": t_batch / a.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched: {len(cfgs)} replicas, K in {{32,48,64,96}}, 8 grains per 16^3, uniaxial "
                               f"0-300 MPa on random axes, kT 0.3-1.0, 26 neighbours, 5^3 zone x 200, refresh every "
                               f"{common.refresh_every}", "sites": sites},
        "replicas_alone": {"value": trials / t_plain, "ms_per_step": t_plain / a.steps * 1e3},
        "batched_over_alone": t_plain / t_batch,
        "autotune": tuned,
        "zone_solve_fraction": st["zone_solves"] / trials,
        "screened": {"value": trials / t_scr, "zone_solve_fraction": st_scr["zone_solves"] / trials},
    }
    print(json.dumps(out), flush=True)


def bench_adjoint(a):
    """Forward (cold start + 2000 explicit steps, checkpoint every 50) and backward of the
    stored elastic energy on the 64^3 / 500-grain workload."""
    import numpy as np
    import torch

    from paper_1009_0457_amd import hmc as H
    from paper_1009_0457_amd.synth import adjoint_config

    micro, sig, probe = adjoint_config()
    K = micro.K
    p = H.hmc_default_params(K, 26, 2)
    p.refresh_tile_z = a.tile_z
    lat = H.Lattice(p, micro.Q)
    lat.set_orientations(micro.euler)
    lat.set_spins(micro.spins)
    lat.set_load(sig)
    lat.elastic_forward(2000, 50)          # warm-up (allocates the adjoint workspace)
    lat.elastic_backward(1.0)
    tf, tb = [], []
    for _ in range(max(1, a.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        U = lat.elastic_forward(2000, 50)
        t1 = time.perf_counter()
        ge, gs = lat.elastic_backward(1.0)
        t2 = time.perf_counter()
        tf.append(t1 - t0)
        tb.append(t2 - t1)
    # The plain method on the same GPU: central differences of the forward for the probe
    # grains' angles (h = 1e-2 rad: the FP32 forward's rounding makes smaller steps noisy).
    h = 1e-2
    fd_abs = []
    n_fwd = 0
    t_fd0 = time.perf_counter()
    for g in probe:
        for k in range(3):
            u_pm = []
            for sgn in (1.0, -1.0):
                e = micro.euler.copy()
                e[g, k] += sgn * h
                lat.set_orientations(e)
                u_pm.append(lat.elastic_forward(2000, 50))
                n_fwd += 1
            fd_abs.append(abs((u_pm[0] - u_pm[1]) / (2 * h) - ge[g, k]))
    t_fd = (time.perf_counter() - t_fd0) / n_fwd
    lat.set_orientations(micro.euler)
    n_params = 3 * micro.Q + 6
    plain = {"method": "central differences of the GPU forward", "h_rad": h, "angles_checked": len(fd_abs),
             "max_abs_diff_over_max_grad": float(max(fd_abs) / np.abs(ge).max()),
             "seconds_per_forward": t_fd, "full_gradient_s": 2 * n_params * t_fd,
             "adjoint_speedup": 2 * n_params * t_fd * (1.0 / (float(np.median(tf)) + float(np.median(tb))))}
    log(f"[bench] plain FD: {plain}")
    lat.set_profiling(True)
    lat.kernel_times()
    lat.elastic_forward(2000, 50)
    kf = lat.kernel_times()
    lat.elastic_backward(1.0)
    kb = lat.kernel_times()
    lat.close()
    f, bk = float(np.median(tf)), float(np.median(tb))
    step_bytes = REFRESH_BYTES_PER_NODE_STEP * K ** 3
    fs = kf["refresh_step"]
    out = {
        "metric": "forward+backward of dU/d(Euler angles, load) per second (64^3, 2000 steps, checkpoint 50)",
        "value": 1.0 / (f + bk), "unit": "gradients/s", "n_gpus": 1, "steps": len(tf), "warmup": 1,
        "ms_per_step": (f + bk) * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"adjoint: {K}^3, {micro.Q} grains, 6 stress components U(+-200 MPa), 2000 explicit "
                               f"steps, checkpoint every 50"},
        "tile_z": a.tile_z,
        "forward_s": f, "backward_s": bk, "backward_over_forward": bk / f, "U": U,
        "forward_step_GBs": step_bytes * fs["launches"] / (fs["total_ms"] * 1e-3) / 1e9 if fs["launches"] else None,
        "adjoint_step_ms": kb["refresh_step"]["total_ms"] / max(1, kb["refresh_step"]["launches"]),
        "forward_step_ms": fs["total_ms"] / max(1, fs["launches"]),
        "plain_method": plain,
    }
    print(json.dumps(out), flush=True)


def big_lattice(a, default_K=512):
    """The large workload's grain structure on a bigger lattice (K a multiple of 128: each
    128^3 Voronoi site refined into a block), for bandwidth measurements beyond the caches."""
    return big_lattice_of(a.K or default_K)


def big_lattice_of(K):
    from paper_1009_0457_amd.synth import large_config, refined_polycrystal, voronoi_polycrystal

    cfg = large_config()
    if K % cfg.K == 0:
        micro = refined_polycrystal(K, K // cfg.K, cfg.n_grains, cfg.seed)
    else:
        micro = voronoi_polycrystal(K, max(8, cfg.n_grains * K ** 3 // cfg.K ** 3), cfg.seed)
    return cfg, K, micro


def measure_potts(cfg, K, micro, proposal, steps, warmup):
    """Zero-load sweeps with kernel timing on: (elapsed s, statistics, colour-pass roofline)."""
    import numpy as np
    import torch

    from paper_1009_0457_amd import hmc as H

    p = H.hmc_default_params(K, cfg.neighbors, cfg.zone_h)
    p.kT = cfg.kT
    p.proposal = 0 if proposal == "neighbor" else 1
    p.seed = cfg.philox_seed
    lat = H.Lattice(p, micro.Q)
    lat.set_orientations(micro.euler)
    lat.set_spins(micro.spins)
    lat.set_load(np.zeros(6))
    for _ in range(warmup):
        lat.sweep(1)
    torch.cuda.synchronize()
    lat.reset_stats()
    lat.kernel_times()
    lat.set_profiling(True)
    t0 = time.perf_counter()
    lat.sweep(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    lat.set_profiling(False)
    kt = lat.kernel_times()["potts"]
    st = lat.stats()
    lat.close()
    colours = 8 if p.neighbors == 26 else 2
    bytes_pass = (2 * colours + 2) * K ** 3 / colours
    ms = kt["total_ms"] / max(1, kt["launches"])
    ach = bytes_pass / (ms * 1e-3) / 1e9
    tr = measured_traffic("potts512_pass_traffic_bytes_per_launch", "potts_source_sha256_16", "hmc_potts.hip",
                          "bandwidth512.md") if K == 512 else None
    roof = {"kernel": "colour pass", "bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": None if tr is None else round(tr),
            "avg_launch_ms": round(ms, 4), "launches": kt["launches"],
            "note": f"(2C+2) bytes of spins per site-trial; lattice {2 * K ** 3 / 2 ** 20:.0f} MiB"}
    return el, st, roof


def bench_potts(a):
    """Zero-load colour passes (integer thresholds decide inside the pass) on a lattice whose
    spins (2 B per site) exceed the 256 MB Infinity Cache."""
    cfg, K, micro = big_lattice(a)
    log(f"[bench] potts: {K}^3, {micro.Q} grains, zero load")
    el, st, roof = measure_potts(cfg, K, micro, a.proposal, a.steps, a.warmup)
    out = {"metric": "site-trials/sec at zero load (colour passes, integer Metropolis thresholds)",
           "value": a.steps * K ** 3 / el, "unit": "site-trials/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": el / a.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "int16", "data": "synthetic",
           "config": {"workload": f"potts-{K}: {K}^3 periodic, 26 neighbours / 8 colours, the 128^3 4000-grain "
                                  f"Voronoi structure refined x{K // 128 if K % 128 == 0 else 1}, no load, kT {cfg.kT}, "
                                  f"proposal {a.proposal}", "K": K},
           "roofline": roof,
           "real_flip_fraction": st["real_flips"] / max(1, st["site_trials"]),
           "acceptance": st["accepted"] / max(1, st["real_flips"])}
    print(json.dumps(out), flush=True)


def bench_growth(a):
    """Sec. 6's grain-growth study: ten independent 60^3 runs, 99 orientations, random spins,
    kT/J = 1.0, zero load, as one fused batch with graph-replayed sweeps; against the same
    runs one after another as single lattices, and the oracle's sweeps on one run."""
    import numpy as np
    import torch

    from paper_1009_0457_amd import hmc as H
    from paper_1009_0457_amd.synth import haar_euler, random_spins

    K, Q, runs = 60, 99, 10
    M = 26 if a.neighbors is None else a.neighbors
    colours = 8 if M == 26 else 2
    common = H.hmc_default_params(K, M, 1)
    common.proposal = 0 if a.proposal == "neighbor" else 1
    reps, init = [], []
    for r in range(runs):
        rep = H.hmc_default_replica(common, K, Q)
        rep.kT, rep.lambda_el, rep.seed = 1.0, 0.0, 9000 + r
        reps.append(rep)
        init.append((haar_euler(np.random.default_rng(8000 + r), Q), random_spins(K, Q, 7000 + r)))
    log(f"[bench] growth: {runs} x {K}^3, Q={Q}, {M} neighbours, kT/J=1.0, zero load")

    def fresh_batch():
        b = H.Batch(common, reps)
        for r, (eu, q0) in enumerate(init):
            b.set_replica(r, eu, q0)
        return b

    # kernel duration of the colour pass (profiling bypasses the graphs), from the initial state
    b = fresh_batch()
    for _ in range(a.warmup):
        b.sweep(1)
    b.synchronize()
    b.kernel_times()
    b.set_profiling(True)
    b.sweep(a.steps)
    b.synchronize()
    b.set_profiling(False)
    kt = b.kernel_times()["potts"]
    b.close()
    # timed: graph-replayed sweeps of the whole batch
    b = fresh_batch()
    b.set_graphs(True)
    for _ in range(a.warmup):
        b.sweep(1)
    b.synchronize()
    b.reset_stats()
    t0 = time.perf_counter()
    b.sweep(a.steps)
    b.synchronize()
    t_batch = time.perf_counter() - t0
    st = b.stats()
    # the grain-size measurement of every run on the GPU (hmc_grain_labels)
    t0 = time.perf_counter()
    n_grains = [b.grain_labels(r)[1] for r in range(runs)]
    t_labels = time.perf_counter() - t0
    b.close()
    # the same runs one after another
    t_plain = 0.0
    for r, (eu, q0) in enumerate(init):
        p = H.hmc_params.from_buffer_copy(common)
        p.kT, p.lambda_el, p.seed = 1.0, 0.0, reps[r].seed
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            lat = H.Lattice(p, Q, stream=s)
            lat.set_orientations(eu)
            lat.set_spins(q0)
            lat.set_graphs(True)
            for _ in range(a.warmup):
                lat.sweep(1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lat.sweep(a.steps)
            s.synchronize()
            t_plain += time.perf_counter() - t0
            lat.close()
    sites = runs * K ** 3
    trials = sites * a.steps
    ms = kt["total_ms"] / max(1, kt["launches"])
    bytes_pass = (2 * colours + 2) * sites / colours
    ach = bytes_pass / (ms * 1e-3) / 1e9
    log(f"[bench] batch {t_batch:.3f} s, runs alone {t_plain:.3f} s, colour pass {ms * 1e3:.1f} us")
    out = {"metric": "site-trials/sec at zero load (grain growth, fused batch of runs)",
           "value": trials / t_batch, "unit": "site-trials/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": t_batch / a.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "int16", "data": "synthetic",
           "config": {"workload": f"growth: {runs} runs of {K}^3, {Q} orientations, random spins, {M} neighbours / "
                                  f"{colours} colours, kT/J 1.0, zero load, proposal {a.proposal}", "sites": sites},
           "roofline": {"kernel": "colour pass", "bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS,
                        "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": None,
                        "avg_launch_ms": round(ms, 4),
                        "note": f"(2C+2) bytes of spins per site-trial over all {runs} runs; "
                                f"{2 * sites / 2 ** 20:.1f} MiB of spins, cache-resident"},
           "runs_alone": {"value": trials / t_plain, "ms_per_step": t_plain / a.steps * 1e3},
           "batched_over_alone": t_plain / t_batch,
           "grain_count_ms_per_run": round(t_labels / runs * 1e3, 3),
           "mean_grain_volume": K ** 3 * runs / float(sum(n_grains)),
           "real_flip_fraction": st["real_flips"] / max(1, st["site_trials"]),
           "acceptance": st["accepted"] / max(1, st["real_flips"])}
    if not a.no_cpu_baseline:
        import oracle as O

        eu, q = init[0]
        q = q.copy()
        prm = O.make_params(K, M, Q, proposal=common.proposal, elastic=False, J=common.J, kT=1.0,
                            seed=reps[0].seed)
        d = np.zeros(1)
        Ct = np.zeros(36 * Q)
        n, t_cpu, s0 = 0, 0.0, 0
        while t_cpu < 10.0 and n < 400:
            t0 = time.perf_counter()
            O.sweeps(prm, q, Ct, Ct, d, np.zeros(6), d, s0, 1)
            t_cpu += time.perf_counter() - t0
            s0 += 1
            n += 1
        out["cpu_baseline"] = {"value": n * K ** 3 / t_cpu, "unit": "site-trials/s", "cores": 1, "kind": "oracle",
                               "sample": f"the oracle's checkerboard sweeps 0..{n - 1} of run 0 ({t_cpu:.1f} s); "
                                         f"serial C, -O2"}
    print(json.dumps(out), flush=True)


def bench_texture(a):
    """Sec. 7's experiment: ten 100^3 runs of 91 rotations about z as one batch; coarsening
    (untimed), then the timed loaded phase of 75 sub-loads to 30 MPa along x, each a warm
    200-step refresh (2000-step cold start at the first) and one sweep with the decision-exact
    zone screen.  A step is one sub-load."""
    import numpy as np

    from paper_1009_0457_amd import texture as T

    K, runs, substeps = 100, 10, 75
    log(f"[bench] texture: {runs} x {K}^3, 91 orientations about z, 30 MPa in {substeps} sub-loads")
    mp = 8 if a.material_points == 8 else 1
    out_run = T.texture_run(K, runs, substeps=substeps, record_every=substeps, profile=True, tile_z=a.tile_z,
                            material_points=mp)
    wall = out_run["wall_s"]
    kt = out_run["kernel_times"]
    st = out_run["stats"]
    trials = runs * K ** 3 * substeps
    ks = kt["refresh_step"]
    ms = ks["total_ms"] / max(1, ks["launches"])
    node_steps = runs * K ** 3
    per_site = 268.0 / 8 if mp == 8 else 50.0
    ach = per_site * node_steps / (ms * 1e-3) / 1e9
    PHI = np.arange(91.0)
    F0, F1 = out_run["fractions"][0].mean(0), out_run["fractions"][-1].mean(0)
    log(f"[bench] loaded phase {wall:.2f} s; explicit step {ms * 1e3:.1f} us x {ks['launches']}")
    out = {"metric": "site-trials/sec of the loaded texture run (sub-load refresh + sweep, zone solves screened)",
           "value": trials / wall, "unit": "site-trials/s", "n_gpus": 1, "steps": substeps, "warmup": 0,
           "ms_per_step": wall / substeps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"texture: {runs} runs of {K}^3, 91 rotations about z, coarsened 100 sweeps at "
                                  f"kT/J 2.6, 30 MPa xx in {substeps} sub-loads (refresh 200 steps, cold 2000, then "
                                  f"one sweep), 26 neighbours, 5^3 zone x 200, screen on"
                                  + (", 2x2x2 material points per cell" if mp == 8 else ""), "sites": runs * K ** 3,
                      "tile_z": a.tile_z, "material_points": mp},
           "roofline": {"kernel": "explicit step", "bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS,
                        "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": None,
                        "avg_launch_ms": round(ms, 4),
                        "note": f"{per_site} B per site-step (the explicit step's algorithmic bytes) over all runs"},
           "kernel_ms": {k: round(v["total_ms"], 2) for k, v in kt.items()},
           "zone_solve_fraction": st["zone_solves"] / trials,
           "texture": {"soft10_before": T.soft_fraction(PHI, F0), "soft10_after": T.soft_fraction(PHI, F1),
                       "mean_abs_dev_before": T.mean_abs_deviation(PHI, F0),
                       "mean_abs_dev_after": T.mean_abs_deviation(PHI, F1)}}
    if not a.no_cpu_baseline:
        import oracle as O
        from paper_1009_0457_amd.synth import texture_run_inputs

        eu, q = texture_run_inputs(K, 1)[0]
        Ct, St, _ = O.tables(eu, 250.8, 150.0, 123.5)
        from paper_1009_0457_amd import hmc as H

        p = H.hmc_default_params(K, 26, 2)
        t0 = time.perf_counter()
        u, E, sig, _ = O.global_solve(K, q, Ct, St, np.array([30.0, 0, 0, 0, 0, 0]) * 1e-3, 1, True, p.glob_alpha,
                                      p.glob_beta, p.glob_alphaE)
        t_step = time.perf_counter() - t0
        prm = O.make_params(K, 26, 91, proposal=0, h=2, nr=200, elastic=True, J=1.0, kT=2.6,
                            lambda_el=p.lambda_el, zone_alpha=p.zone_alpha, zone_beta=p.zone_beta,
                            Sigma=(0.03, 0, 0, 0, 0, 0), seed=400)
        g = np.arange(K)
        z, y, x = np.meshgrid(g, g, g, indexing="ij")
        sites = np.nonzero((((x | y | z) & 1) == 0).ravel())[0]
        np.random.default_rng(5).shuffle(sites)
        done, t_tr, batch = 0, 0.0, 64
        while t_tr < a.cpu_seconds and done < sites.size:
            pick = sites[done:done + batch]
            t0 = time.perf_counter()
            O.trials(prm, q, Ct, St, sig, 0, pick)
            t_tr += time.perf_counter() - t0
            done += pick.size
            batch = min(4096, batch * 2)
        t_sub = 200 * t_step + K ** 3 * t_tr / done
        out["cpu_baseline"] = {"value": K ** 3 / t_sub, "unit": "site-trials/s", "cores": 1, "kind": "oracle",
                               "sample": f"{done} random site-trials of colour pass 0 on run 0's random start "
                                         f"({t_tr:.1f} s) + 1 explicit step at {K}^3 ({t_step:.1f} s), combined as "
                                         f"K^3 trials + 200 steps per sub-load; serial FP64 C, -O2"}
    print(json.dumps(out), flush=True)


def measure_refresh(cfg, K, micro, n, warm, tile_z=0, mp8=False):
    """Warm explicit steps with kernel timing on: (elapsed s, explicit-step roofline, fold ms)."""
    import torch

    from paper_1009_0457_amd import hmc as H

    p = H.hmc_default_params(K, cfg.neighbors, cfg.zone_h)
    p.refresh_tile_z = tile_z
    if mp8:
        H.hmc_set_material_points(p, 8)
    lat = H.Lattice(p, micro.Q)
    lat.set_orientations(micro.euler)
    lat.set_spins(micro.spins)
    lat.set_load(cfg.sigma_MPa)
    lat.stress_refresh(max(1, warm), True)
    torch.cuda.synchronize()
    lat.kernel_times()
    lat.set_profiling(True)
    t0 = time.perf_counter()
    lat.stress_refresh(n, False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    lat.set_profiling(False)
    kt = lat.kernel_times()
    lat.close()
    ks = kt["refresh_step"]
    ms = ks["total_ms"] / max(1, ks["launches"])
    # 8 points per cell, per cell and step: corner displacements 12 B (each node once), 8 spins
    # 16 B, 24 corner forces written 96 B and read back 96 B, u and w read and written 48 B
    per_site = 268.0 / 8 if mp8 else REFRESH_BYTES_PER_NODE_STEP
    ach = per_site * K ** 3 / (ms * 1e-3) / 1e9
    tr = measured_traffic("refresh512_step_traffic_bytes_per_launch", "elastic_source_sha256_16", "hmc_elastic.hip",
                          "bandwidth512.md") if (K == 512 and not mp8 and tile_z == 0) else None
    roof = {"kernel": "global explicit step", "bound": "hbm", "achieved": round(ach, 1),
            "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4),
            "traffic": None if tr is None else round(tr), "avg_launch_ms": round(ms, 4), "launches": ks["launches"],
            "note": (f"{per_site} B per site-step (cell pass, node pass and E fold)" if mp8 else
                     f"50 B per node-step; working set {(13 * 4 + 2) * K ** 3 / 2 ** 30:.2f} GiB")}
    fold = round(kt["refresh_other"]["total_ms"] / max(1, kt["refresh_other"]["launches"]), 4)
    return el, roof, fold


def bench_refresh(a):
    """Explicit global steps (Sec. 5 relaxation) on a lattice whose 54 B/site working set
    exceeds the 256 MB Infinity Cache."""
    cfg, K, micro = big_lattice(a)
    n = a.steps * 10
    mp8 = a.material_points == 8
    log(f"[bench] refresh: {K}^3, {micro.Q} grains, {n} steps")
    el, roof, fold = measure_refresh(cfg, K, micro, n, a.warmup * 10, a.tile_z, mp8)
    out = {"metric": "explicit global stress-refresh steps/sec", "value": n / el, "unit": "steps/s", "n_gpus": 1,
           "steps": n, "warmup": a.warmup * 10, "ms_per_step": el / n * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"refresh-{K}: {K}^3 periodic, the 128^3 4000-grain Voronoi structure refined "
                                  f"x{K // 128 if K % 128 == 0 else 1}, biaxial 150/150 MPa, warm steps"
                                  + (", 2x2x2 material points per cell of 2^3 sites" if mp8 else ""), "K": K,
                      "tile_z": a.tile_z, "material_points": 8 if mp8 else 1},
           "roofline": roof,
           "fold_ms": fold}
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; sharding over several GPUs is not implemented",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    if a.copy_probe_mib:
        import torch

        src = torch.ones(a.copy_probe_mib * 2 ** 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {a.copy_probe_mib} MiB read + {a.copy_probe_mib} MiB written")
        del src, dst
    if a.workload == "batched":
        return bench_batched(a)
    if a.workload == "adjoint":
        return bench_adjoint(a)
    if a.workload == "potts":
        return bench_potts(a)
    if a.workload == "refresh":
        return bench_refresh(a)
    if a.workload == "growth":
        return bench_growth(a)
    if a.workload == "texture":
        return bench_texture(a)
    import numpy as np
    import torch

    from paper_1009_0457_amd import hmc as H
    from paper_1009_0457_amd.synth import large_config, voronoi_polycrystal

    cfg = large_config()
    if a.zero_load:
        cfg = cfg.zero_load()
    K = a.K or cfg.K
    log(f"[bench] building {K}^3 microstructure with {cfg.n_grains} grains")
    micro = voronoi_polycrystal(K, cfg.n_grains if K == cfg.K else max(8, cfg.n_grains * K ** 3 // cfg.K ** 3),
                                cfg.seed)
    zh = cfg.zone_h if a.zone_h is None else a.zone_h
    p = H.hmc_default_params(K, cfg.neighbors, zh)
    p.kT = cfg.kT
    p.zone_steps = cfg.zone_steps if a.zone_steps is None else a.zone_steps
    p.refresh_every = cfg.refresh_every
    p.proposal = 0 if a.proposal == "neighbor" else 1
    p.seed = cfg.philox_seed
    p.zone_variant = a.zone_variant
    p.refresh_tile_z = a.tile_z
    # the library's own stream, so that sweeps are captured into HIP graphs and replayed
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    lat = H.Lattice(p, micro.Q, stream=stream)
    lat.set_orientations(micro.euler)
    lat.set_spins(micro.spins)
    lat.set_load(cfg.sigma_MPa)
    if not a.zero_load:
        log(f"[bench] cold refresh ({p.cold_steps} steps)")
        lat.stress_refresh(-1, True)
    lat.synchronize()
    # The timed region runs with kernel timing on (a pair of HIP events on the library's
    # stream around every launch), which launches eagerly; the same sweeps replayed from HIP
    # graphs without timing follow as a second figure.
    lat.set_profiling(True)
    log(f"[bench] warmup {a.warmup} sweeps")
    for _ in range(a.warmup):
        lat.sweep(1)
    lat.synchronize()
    lat.reset_stats()
    lat.kernel_times()
    axes = [ax for ax in cfg.histogram_axes]
    hist = []
    log(f"[bench] timing {a.steps} sweeps")
    lat.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        s = lat.sweep_index()
        lat.sweep(1)
        if cfg.histogram_every and (s + 1) % cfg.histogram_every == 0:
            hist.append([lat.texture_histogram(ax, 10.0, 6).tolist() for ax in axes])
    lat.synchronize()
    t1 = time.perf_counter()
    kt = lat.kernel_times()
    lat.set_profiling(False)
    st = lat.stats()
    elapsed = t1 - t0
    trials = a.steps * K ** 3
    value = trials / elapsed
    log(f"[bench] {elapsed:.3f} s, {value:.4e} site-trials/s, stats {st}")

    solves = st["zone_solves"]
    zt = kt["zone"]
    fps = zone_flops_per_solve(p.zone_h, p.zone_steps)
    zsec = zt["total_ms"] * 1e-3
    achieved = fps * solves / zsec / 1e12 if zsec > 0 else 0.0
    workload_zone = (p.zone_h, p.zone_steps) == (2, 200)   # the zone the counters were taken on
    per_solve = measured_traffic("zone_traffic_bytes_per_solve", "zone_source_sha256_16",
                                 ZONE_H2_SOURCES) if workload_zone else None
    spl = solves / max(1, zt["launches"])
    roof = {"kernel": "zone solve", "bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "traffic": None if per_solve is None else round(per_solve * spl),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE, profiles/counters_large128.md)",
            "avg_launch_ms": round(zt["total_ms"] / max(1, zt["launches"]), 4),
            "flop_per_solve": fps, "solves_per_launch": round(solves / max(1, zt["launches"]), 1)}
    # the same launches priced at the least work of the kernels' separable form and at the FP32
    # operations the kernel executes (its VALU counters, lanes without a voxel included)
    mfps = zone_flops_minimal(p.zone_h, p.zone_steps)
    roof["flop_per_solve_minimal"] = mfps
    roof["frac_minimal"] = round(mfps * solves / zsec / 1e12 / PEAK_FP32_TFLOPS, 4) if zsec > 0 else None
    xfps = measured_traffic("zone_executed_fp32_flop_per_solve", "zone_source_sha256_16", ZONE_H2_SOURCES,
                            "zone_instruction_mix_large128.md") if workload_zone else None
    roof["flop_per_solve_executed"] = xfps
    roof["frac_executed"] = round(xfps * solves / zsec / 1e12 / PEAK_FP32_TFLOPS, 4) if (xfps and zsec > 0) else None
    pk = kt["potts"]
    potts_roof = None
    if pk["launches"]:
        colours = 8 if p.neighbors == 26 else 2
        bytes_pass = (2 * colours + 2) * K ** 3 / colours      # (2C+2) B per site-trial of the class
        ach = bytes_pass * pk["launches"] / (pk["total_ms"] * 1e-3) / 1e9
        potts_roof = {"kernel": "colour pass", "bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS,
                      "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4),
                      "avg_launch_ms": round(pk["total_ms"] / pk["launches"], 4),
                      "note": "(2C+2) bytes of spins per site-trial (the lattice read once per pass)"}
    rs = kt["refresh_step"]
    refresh_roof = None
    if rs["launches"]:
        bytes_step = REFRESH_BYTES_PER_NODE_STEP * K ** 3
        ach = bytes_step * rs["launches"] / (rs["total_ms"] * 1e-3) / 1e9
        rt = measured_traffic("refresh_step_traffic_bytes_per_launch", "elastic_source_sha256_16", "hmc_elastic.hip")
        refresh_roof = {"kernel": "global explicit step", "bound": "hbm", "achieved": round(ach, 1),
                        "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4),
                        "traffic": None if (rt is None or K != 128) else round(rt),
                        "avg_launch_ms": round(rs["total_ms"] / rs["launches"], 4),
                        "note": f"working set {(13 * 4 + 2) * K ** 3 / 2 ** 20:.0f} MiB (cache-resident at 128^3)"}
    out = {
        "metric": METRIC if p.zone_h == 2 else METRIC.replace("5^3 zone", f"{2 * p.zone_h + 1}^3 zone"),
        "value": value,
        "unit": "site-trials/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": elapsed / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"large-{K}: {K}^3 periodic, 26 neighbours / 8 colours, {micro.Q} Voronoi grains, "
                               f"{'no load (elastic term off)' if a.zero_load else 'biaxial 150/150 MPa'}, kT {p.kT}, "
                               f"{2 * p.zone_h + 1}^3 zone x {p.zone_steps} steps, refresh every "
                               f"{p.refresh_every} sweeps x {p.refresh_steps} steps, proposal {a.proposal}",
                   "K": K, "neighbors": p.neighbors, "zone_h": p.zone_h, "zone_steps": p.zone_steps,
                   "proposal": a.proposal, "zone_variant": a.zone_variant},
        "zone_solve_fraction": solves / trials,
        "zone_solves_per_s": solves / elapsed,
        "acceptance": st["accepted"] / max(1, st["real_flips"]),
        "roofline": roof,
        "refresh_roofline": refresh_roof,
        "potts_roofline": potts_roof,
        "kernel_ms": {k: round(v["total_ms"], 3) for k, v in kt.items()},
    }
    # the same sweeps replayed from HIP graphs (one graph per sweep), kernel timing off
    lat.set_graphs(True)
    lat.sweep(2)                                  # capture both sweep graphs
    lat.synchronize()
    lat.reset_stats()
    tg0 = time.perf_counter()
    for _ in range(a.steps):
        s = lat.sweep_index()
        lat.sweep(1)
        if cfg.histogram_every and (s + 1) % cfg.histogram_every == 0:
            hist.append([lat.texture_histogram(ax, 10.0, 6).tolist() for ax in axes])
    lat.synchronize()
    tg = time.perf_counter() - tg0
    stg = lat.stats()
    lat.set_graphs(False)
    out["graph_replayed"] = {"value": trials / tg, "unit": "site-trials/s", "ms_per_step": tg / a.steps * 1e3,
                             "zone_solve_fraction": stg["zone_solves"] / trials,
                             "note": "the next sweeps of the same run, each replayed from a captured HIP graph "
                                     "(kernel timing off)"}
    log(f"[bench] graph-replayed: {trials / tg:.4e} site-trials/s")
    if a.zero_load:
        lat.close()
        print(json.dumps(out), flush=True)
        return
    # the same workload with the lower-bound screen (decision-exact; fewer zone solves)
    lat.set_zone_screen(True)
    lat.reset_stats()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(a.steps):
        s = lat.sweep_index()
        lat.sweep(1)
        if cfg.histogram_every and (s + 1) % cfg.histogram_every == 0:
            hist.append([lat.texture_histogram(ax, 10.0, 6).tolist() for ax in axes])
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    st2 = lat.stats()
    lat.set_zone_screen(False)
    out["screened"] = {
        "value": trials / (t3 - t2), "unit": "site-trials/s", "ms_per_step": (t3 - t2) / a.steps * 1e3,
        "zone_solve_fraction": st2["zone_solves"] / trials, "screened_fraction": st2["screened"] / trials,
        "note": "same workload and sweep count, zone_screen=1: trials whose point-zone lower bound already "
                "exceeds the Metropolis threshold are rejected without a solve (decisions unchanged)"}
    log(f"[bench] screened: {out['screened']['value']:.4e} site-trials/s, stats {st2}")
    if a.proposal == "neighbor" and a.saturation_steps > 0:
        out["saturation_uniform"] = saturation_line(a, p, micro, lat, cfg)
    if not a.no_cpu_baseline:
        log("[bench] oracle CPU baseline")
        out["cpu_baseline"] = cpu_baseline(lat, p, micro, a.cpu_seconds)
        lat.close()
        out["cpu_baseline"]["small_configs"] = small_configs()
    else:
        lat.close()
    if a.bandwidth_K:
        out["beyond_caches"] = bandwidth_leg(a.bandwidth_K)
    print(json.dumps(out), flush=True)


def bandwidth_leg(K):
    """The two bandwidth-bound kernels on the large workload's grain structure refined to K^3
    (512^3: 256 MiB of spins and 6.75 GiB of explicit-step arrays, beyond the 256 MB Infinity
    Cache): zero-load colour passes and warm explicit steps, kernel timing on."""
    cfg, K, micro = big_lattice_of(K)
    log(f"[bench] beyond the caches: {K}^3 colour passes and explicit steps")
    sweeps, steps = 10, 40
    _, st, potts = measure_potts(cfg, K, micro, "neighbor", sweeps, 2)
    _, step, _ = measure_refresh(cfg, K, micro, steps, 20)
    return {"workload": f"{K}^3 periodic, the 128^3 4000-grain Voronoi structure refined x{K // 128}, 26 neighbours / "
                        f"8 colours: {sweeps} zero-load sweeps, then {steps} warm explicit steps under biaxial 150/150 MPa",
            "colour_pass": potts, "explicit_step": step,
            "real_flip_fraction": st["real_flips"] / max(1, st["site_trials"])}


def saturation_line(a, p, micro, lat, cfg):
    """The same lattice state (spins, stress field and displacements after the timed sweeps)
    with uniform proposals: every trial is a real flip and gets a zone solve (f_z = 1), which
    loads the zone kernel fully; a few sweeps with kernel timing on."""
    from paper_1009_0457_amd import hmc as H

    q = H.hmc_params.from_buffer_copy(p)
    q.proposal = 1
    u = H.Lattice(q, micro.Q, stream=lat.stream)
    u.set_orientations(micro.euler)
    u.set_spins(lat.get_spins())
    u.set_load(cfg.sigma_MPa)
    u.set_elastic_state(lat.get_displacement(), lat.macro_strain())
    u.stress_refresh(0, False)
    u.set_sweep_index(lat.sweep_index())
    u.set_profiling(True)
    u.sweep(1)
    u.synchronize()
    u.reset_stats()
    u.kernel_times()
    n = a.saturation_steps
    t0 = time.perf_counter()
    u.sweep(n)
    u.synchronize()
    el = time.perf_counter() - t0
    kt = u.kernel_times()
    st = u.stats()
    u.close()
    zt = kt["zone"]
    fps = zone_flops_per_solve(q.zone_h, q.zone_steps)
    ach = fps * st["zone_solves"] / (zt["total_ms"] * 1e-3) / 1e12 if zt["total_ms"] > 0 else 0.0
    log(f"[bench] uniform proposals: {n * q.K ** 3 / el:.4e} site-trials/s, zone {ach:.1f} TFLOP/s")
    return {"value": n * q.K ** 3 / el, "unit": "site-trials/s", "steps": n, "ms_per_step": el / n * 1e3,
            "zone_solve_fraction": st["zone_solves"] / (n * q.K ** 3), "zone_solves_per_s": st["zone_solves"] / el,
            "zone_roofline": {"achieved": round(ach, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                              "frac": round(ach / PEAK_FP32_TFLOPS, 4),
                              "frac_minimal": round(ach * zone_flops_minimal(q.zone_h, q.zone_steps) / fps
                                                    / PEAK_FP32_TFLOPS, 4),
                              "avg_launch_ms": round(zt["total_ms"] / max(1, zt["launches"]), 4)},
            "note": "uniform proposals (every trial a real flip, f_z = 1) from the state after the timed sweeps"}


if __name__ == "__main__":
    main()
