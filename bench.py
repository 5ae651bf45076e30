"""Benchmark of the checkerboard Metropolis sweep on one MI355X.

One step is one pass of the whole hot path over one synthetic lattice:
random start (seed 7), acceptance table, 10^3 checkerboard sweeps at
beta = 0.4406868 and a from-scratch recount of E and M, on the L = 4096
lattice with one bit per spin.  The spins live in HBM for the whole run; the
timed region contains only device work launched through the C ABI.

Prints one JSON line: spin-flip attempts per ns (value), the roofline of
the dominant kernel (the persistent tile-resident sweep), and the CPU
oracle timed on the host cores on a bounded sample of the same workload.
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

METRIC = "spin-flip attempts/ns and % HBM roofline; τ_int-normalised samples/s learned vs plain"
BETA = 0.4406868
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, published
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12  # 256 CUs x 64 lanes x 2.4 GHz = 39.3 T lane-ops/s
PHILOX_OPS_PER_BLOCK = 40        # 10 rounds x (2 mul-hi/lo + 2 three-input xor)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--L", type=int, default=4096)
    ap.add_argument("--sweeps", type=int, default=1000)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--layout", choices=("bit1", "int8"), default="bit1",
                    help="single: one bit per spin (default) or one byte per spin")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--global-halfsweep", action="store_true",
                    help="time the one-launch-per-half-sweep kernel instead (same chain)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for HBM counter scaling)")
    ap.add_argument("--workload", choices=("single", "batched", "learned", "ea", "xy", "scaling"),
                    default="single",
                    help="single: one L=4096 bit-packed lattice (default); batched: 1024 INT8 "
                         "lattices of sides 32..256 on a 64-point beta grid in one launch; "
                         "learned: independent samples/s of learned-proposal vs plain chains "
                         "at L=32; ea: 3D +-J spin glass L=128, 64 replicas, replica exchange; "
                         "xy: the paper's XY model at T=0.85, L=8..128, ten seeds; "
                         "scaling: time per sweep against L for both layouts")
    ap.add_argument("--beta", type=float, default=BETA, help="learned: inverse temperature")
    ap.add_argument("--epochs", type=int, default=3, help="learned: training epochs")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched: keep the library's default launch shape")
    ap.add_argument("--draws", choices=("plane", "site"), default="plane",
                    help="batched and ea: bit-plane draws (32 sites per lane) or per-site draws")
    ap.add_argument("--shape", default=None,
                    help="batched: launch shape THREADS,GROUPS_PER_CU instead of autotuning")
    return ap.parse_args()


# Sources whose text determines each profiled sweep kernel's code.
KERNEL_SOURCES = {
    "bit1_kernels.hip": ("bit1_kernels.hip", "common.hpp", "kernels.hpp", "bitslice.hpp",
                         "handoff.hpp"),
    "batch_kernels.hip": ("batch_kernels.hip", "common.hpp", "kernels.hpp", "batch.hpp", "quad.hpp"),
    "ea_kernels.hip": ("ea_kernels.hip", "common.hpp", "kernels.hpp", "ea.hpp", "bitslice.hpp"),
    "batch_bit_kernels.hip": ("batch_bit_kernels.hip", "common.hpp", "kernels.hpp", "batch.hpp",
                              "bitslice.hpp"),
}


def kernel_source_hash(source: str) -> str:
    """sha256 over the sources that determine the kernels of `source`."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[source]:
        h.update(open(os.path.join(ROOT, "paper_2402_06415_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def profiled_traffic(kernel_name: str, summary: str = "sweep_bit1_L4096",
                     source: str = "bit1_kernels.hip"):
    """HBM bytes per launch of a sweep kernel from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE, scaled by a 1 GiB copy), or
    None when the kernel sources have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{summary}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel") != kernel_name or \
            rec.get("kernel_source_sha256") != kernel_source_hash(source):
        return None
    return rec


def bit1_sweep_kernel(L: int, cus: int) -> str:
    """Name of the kernel the library's bit-packed sweep of side L runs,
    by the host-side rule of its tile plan: rows of at most 64 words take
    one tile per CU of up to 16 rows, one wave per row, draws pipelined
    (k_sweep_bit1_rows_pipe); wider rows up to four tiles per CU that each
    fit a share of the CU's LDS (one wave per row: k_sweep_bit1_rows,
    several: k_sweep_bit1_tiles); lattices whose tiles do not fit run one
    launch per half-sweep (k_halfsweep_bit1)."""
    nw = L >> 6
    if nw < 1 or cus < 1:
        return "k_halfsweep_bit1"
    if nw <= 64:
        return "k_sweep_bit1_rows_pipe"
    tpc = 4 if L >= 16 * cus else 1
    cap = min(160 * 1024 // tpc, 64 * 1024)
    fits = [t for t in range(min(cus * tpc, 1024, L), 1, -1)
            if L % t == 0 and 2 * (L // t + 2) * nw * 4 <= cap]
    if not fits:
        return "k_halfsweep_bit1"
    best = fits[0]
    best8 = next((t for t in fits if t % 8 == 0), 0)
    if best8 and 2 * best8 >= best:
        best = best8
    rows = L // best
    waves = min(rows, max(16 // tpc, 1))
    return "k_sweep_bit1_rows" if waves == rows else "k_sweep_bit1_tiles"


def valu_ceiling(prof, words_per_launch: int):
    """Attempts/ns the sweep kernel would reach at full VALU issue: the VALU
    lane-operations it spends per 32-site word (rocprofv3 SQ_INSTS_VALU x 64
    lanes / words updated) against the chip's 39.3 T lane-ops/s."""
    if not prof or not prof.get("valu_wave_instructions_per_launch"):
        return None, None
    per_word = prof["valu_wave_instructions_per_launch"] * 64 / words_per_launch
    return per_word, VALU_PEAK_TOPS * 1e12 * 32 / per_word / 1e9


def measured_copy_gbs(torch, dev, nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Read + write bandwidth of a plain device-to-device copy of 1 GiB on
    this GPU (best of a few), the practical ceiling beside the 8 TB/s peak."""
    a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    return 2 * nbytes / (best * 1e-3) / 1e9


def cpu_baseline(L: int, seed: int, target_s: float, layout: str = "bit1"):
    """The oracle (unchanged; plane draws for the bit-packed layout, site
    draws for int8; OpenMP over rows) on a bounded sample: the first sweeps
    of the same lattice from the same start."""
    import oracle

    mode = oracle.MODE_PLANE if layout == "bit1" else oracle.MODE_SITE

    threads = max(1, min(16, os.cpu_count() or 1))
    s = oracle.init(L, oracle.START_RANDOM, seed)
    t0 = time.perf_counter()
    oracle.sweep(s, mode, seed, 0, 0, 1, BETA, record=False, nthreads=threads)
    one = time.perf_counter() - t0
    n = max(1, min(200, int(target_s / max(one, 1e-6))))
    t0 = time.perf_counter()
    oracle.sweep(s, mode, seed, 0, 1, n, BETA, record=False, nthreads=threads)
    dt = time.perf_counter() - t0
    # the same oracle on one core, on the sweeps that follow
    t0 = time.perf_counter()
    oracle.sweep(s, mode, seed, 0, 1 + n, 1, BETA, record=False, nthreads=1)
    one1 = time.perf_counter() - t0
    n1 = max(1, min(20, int(target_s / 3 / max(one1, 1e-6))))
    t0 = time.perf_counter()
    oracle.sweep(s, mode, seed, 0, 2 + n, n1, BETA, record=False, nthreads=1)
    dt1 = time.perf_counter() - t0
    return {
        "value": L * L * n / (dt * 1e9),
        "unit": "spin-flip attempts/ns",
        "cores": threads,
        "kind": "oracle",
        "sample": f"L={L} {'bit-plane' if layout == 'bit1' else 'per-site'} draws, random "
                  f"start seed {seed}, sweeps 1..{n} ({dt:.1f} s), OpenMP over rows of one colour",
        "single_core": {"value": L * L * n1 / (dt1 * 1e9), "cores": 1,
                        "sample": f"sweeps {n + 2}..{n + 1 + n1} of the same chain ({dt1:.1f} s)"},
        "host": host_cpu(),
    }


def host_cpu():
    """Model name and logical CPU count of the host the oracle ran on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count()}


def cpu_baseline_batched(L, beta, seed: int, target_s: float, draws: str = "plane"):
    """The oracle on a bounded sample of the batched workload: the first
    sweeps of the first lattices, each lattice's chain as in the batch."""
    import oracle

    mode = oracle.MODE_PLANE if draws == "plane" else oracle.MODE_SITE
    threads = max(1, min(16, os.cpu_count() or 1))
    m = 64  # lattices in the sample: one full period of the beta grid
    states = [oracle.init(int(L[j]), oracle.START_RANDOM, seed, j) for j in range(m)]
    t0 = time.perf_counter()
    oracle.batch_sweep(states, beta[:m], seed, 0, 0, 1, nthreads=threads, mode=mode)
    one = time.perf_counter() - t0
    n = max(1, min(1000, int(target_s / max(one, 1e-6))))
    t0 = time.perf_counter()
    oracle.batch_sweep(states, beta[:m], seed, 0, 1, n, nthreads=threads, mode=mode)
    dt = time.perf_counter() - t0
    spins = int(sum(int(L[j]) ** 2 for j in range(m)))
    return {
        "value": spins * n / (dt * 1e9),
        "unit": "spin-flip attempts/ns",
        "cores": threads,
        "kind": "oracle",
        "sample": f"lattices 0..{m - 1} of the batch ({spins} spins), sweeps 1..{n} ({dt:.1f} s), "
                  f"{draws} draws, OpenMP over rows (site) or draw groups (plane) of one colour",
    }


def bench_batched(args):
    import torch

    import paper_2402_06415_amd as lib
    from paper_2402_06415_amd.workloads import batched_workload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    seed, nsw = 11, (args.sweeps if args.sweeps != 1000 else 10_000)
    L, beta = batched_workload(seed=seed)
    b = lib.Batch(L, beta, seed=seed, start="random", device=dev, draws=args.draws)
    plane = args.draws == "plane"
    kernel = "k_batch_sweep_bit" if plane else "k_batch_sweep"
    tune = None
    if args.shape:
        b.c.threads, b.c.groups_per_cu = (int(v) for v in args.shape.split(","))
        tune = {"chosen": [int(b.c.threads), int(b.c.groups_per_cu)], "given": True}
    elif not args.no_autotune:
        times = b.autotune(probe_sweeps=200)
        tune = {"chosen": [int(b.c.threads), int(b.c.groups_per_cu)],
                "ms_per_200_sweeps": {f"{t}x{g}": round(ms, 3) for t, g, ms in times}}
    stream = torch.cuda.current_stream()
    mom = torch.zeros((b.count, 8), dtype=torch.int64, device=dev)

    def step():
        b.init("random")
        b.sweep(nsw, out=mom)
        return b.measure()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    b.check()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    sw_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
             for _ in range(args.steps)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for k in range(args.steps):
        b.init("random")
        sw_ev[k][0].record(stream)
        b.sweep(nsw, out=mom)
        sw_ev[k][1].record(stream)
        b.measure()
    ev[1].record(stream)
    torch.cuda.synchronize()
    total_ms = ev[0].elapsed_time(ev[1])
    sweep_ms = sum(a.elapsed_time(c) for a, c in sw_ev) / args.steps
    blocks = b.rng_blocks()
    b.check()
    spins = int((L.astype(np.int64) ** 2).sum())
    attempts = spins * nsw
    ms_per_step = total_ms / args.steps
    achieved_tops = blocks * PHILOX_OPS_PER_BLOCK / (sweep_ms * 1e-3) / 1e12
    alg_bytes = attempts * 2.0  # INT8: read and write each spin once per sweep
    eff_gbs = alg_bytes / (sweep_ms * 1e-3) / 1e9
    prof = (profiled_traffic(kernel, "batch_plane_1024", "batch_bit_kernels.hip") if plane else
            profiled_traffic(kernel, "batch_int8_1024", "batch_kernels.hip")) \
        if nsw == 10_000 else None
    traffic = (prof["hbm_read_bytes_per_launch"] + prof["hbm_write_bytes_per_launch"]) if prof else None
    value = attempts / (ms_per_step * 1e6)
    # plane draws: one 32-site word per lane-update
    valu_per_word, ceiling = valu_ceiling(prof, spins // 32 * nsw) if plane else (None, None)
    rec = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "spin-flip attempts/ns",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {
            "workload": f"1024 independent 2D Ising lattices, sides uniform in {{32,64,128,256}} "
                        f"(seed {seed}), 64-point beta grid in [0.30, 0.60], random starts, "
                        f"{nsw} sweeps in one persistent launch + init + recount per step",
            "lattices": int(b.count), "spins": spins, "sweeps_per_step": nsw, "seed": seed,
            "draws": args.draws,
            "layout": "int8 in HBM, colour bit planes in LDS" if plane else "int8",
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved_tops, 3),
            "peak": round(VALU_PEAK_TOPS, 2),
            "unit": "TOP/s",
            "frac": round(achieved_tops / VALU_PEAK_TOPS, 4),
            "traffic": round(traffic) if traffic else None,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "kernel": kernel,
            "kernel_ms": round(sweep_ms, 4),
            "work": f"{blocks} Philox4x32-10 blocks x {PHILOX_OPS_PER_BLOCK} int ops per launch "
                    "(the blocks the chain needs, counted on a same-chain lattice)",
            "valu_issue_utilisation": round(prof["valu_utilisation"], 3) if prof else None,
            "valu_per_word": round(valu_per_word, 1) if valu_per_word else None,
            "valu_ceiling_attempts_per_ns": round(ceiling, 1) if ceiling else None,
            "frac_of_valu_ceiling": round(value / ceiling, 4) if ceiling else None,
        },
        "hbm_roofline": {
            "achieved": round(eff_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(eff_gbs / HBM_PEAK_GBS, 4),
            "note": "algorithmic 2 B/attempt (INT8 read + write per sweep); lattices stay in LDS",
        },
        "autotune": tune,
    }
    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        c = torch.empty_like(a)
        c.copy_(a)
        torch.cuda.synchronize()
        rec["copy_calibration_bytes"] = 1 << 30
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline_batched(L, beta, seed, args.cpu_seconds, args.draws)
    print(json.dumps(rec), flush=True)


# multiply-adds per site of the proposal network (layers 1-4 of the masked
# network): 64 (mask A, 4 taps x 16) + 2 x 1280 (mask B, 80 x 16) + 80
NN_MAC_PER_SITE = 64 + 2 * 1280 + 80
# the wavefront kernel's products per site and sign: layer 1 as 64 float32
# multiply-adds, layers 2-4 as bfloat16 products with each float32
# activation entering as two bfloat16 terms
NN_WAVE_BF16_MAC_PER_SITE = 2 * (2 * 1280 + 80)
NN_WAVE_F32_MAC_PER_SITE = 64
BF16_MATRIX_PEAK_TFLOPS = 2500.0
# HBM bytes per site of one training step, each pass reading its inputs once
# and writing its outputs once (float32 [B][N][16] activations and gradients,
# 64 bytes a site; int8 spins; float32 dz): forward 65 + 2 x 128 + 69,
# layer 4 backward 68 + 132, layers 3 and 2 backward 2 x (128 + 192),
# layer 1 weight gradient 65
NN_TRAIN_BYTES_PER_SITE = 65 + 2 * 128 + 69 + 68 + 132 + 2 * (128 + 192) + 65
HBM_PEAK_GBS = 8000.0


def bench_learned(args):
    """tau_int-normalised independent samples per second of the chain with
    learned whole-lattice proposals against plain checkerboard sweeps."""
    import torch

    import paper_2402_06415_amd as lib
    from paper_2402_06415_amd.analysis import binned_mean, tau_int
    from paper_2402_06415_amd.learned import LearnedChains, plain_configurations, train
    from paper_2402_06415_amd.workloads import learned_workload, nn_initial_params

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = learned_workload()
    L, chains, k = wl["L"], wl["chains"], wl["sweeps_per_proposal"]
    beta = args.beta
    N = L * L
    stream = torch.cuda.current_stream()

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        out = fn()
        b.record(stream)
        torch.cuda.synchronize()
        return out, a.elapsed_time(b)

    snaps = -(-wl["train_configs"] // chains)  # at least train_configs configurations
    data, gen_ms = timed(lambda: plain_configurations(L, beta, chains, 2000, snaps, 10, seed=101))
    batch = 1024
    net = lib.Net(L, max(batch, chains), params=nn_initial_params(7))
    steps = args.epochs * (data.shape[0] // batch)
    losses, train_ms = timed(lambda: train(net, data, args.epochs, batch, 2e-3, seed=5))
    del data

    # plain chains, equilibrated
    T = 20000
    plain = lib.Batch([L] * chains, [beta] * chains, seed=201, start="random", device=dev)
    plain.autotune()  # the best launch shape for the plain chain too
    plain.sweep(2000, moments=False)
    tr = torch.empty((T, chains, 2), dtype=torch.int64, device=dev)
    _, plain_ms = timed(lambda: plain.sweep(T, moments=False, trace=tr))
    trp = tr.cpu().numpy()
    del tr
    # learned chains
    lc = LearnedChains(net, L, [beta] * chains, seed=301, sweeps_per_proposal=k)
    for _ in range(100):
        lc.cycle()
    cycles = 1000
    tr = torch.empty((cycles * k, chains, 2), dtype=torch.int64, device=dev)
    lc.n_accepted.zero_()

    def run_cycles():
        for c in range(cycles):
            lc.cycle(trace=tr[c * k:(c + 1) * k])

    _, learn_ms = timed(run_cycles)
    trl = tr.cpu().numpy()
    # the dominant kernel of a cycle: the wavefront sampler (the proposals
    # and their log q_sym), timed alone; then the whole-lattice evaluation
    # of log q_sym of the current states
    reps = 20
    prop = torch.empty((chains, L, L), dtype=torch.int8, device=dev)
    lq = torch.empty(chains, dtype=torch.float32, device=dev)
    net.sample(chains, 17, 0, 0, out=prop, logq=lq, symmetric=True)
    _, wave_ms = timed(lambda: [net.sample(chains, 17, 0, d, out=prop, logq=lq, symmetric=True)
                                for d in range(reps)])
    wave_ms /= reps
    net.logq(lc.batch, out=lq, symmetric=True)
    _, lattice_ms = timed(lambda: [net.logq(lc.batch, out=lq, symmetric=True) for _ in range(reps)])
    lattice_ms /= reps
    nn_flop = chains * 2 * N * (NN_WAVE_BF16_MAC_PER_SITE + NN_WAVE_F32_MAC_PER_SITE) * 2
    wave_tflops = nn_flop / (wave_ms * 1e-3) / 1e12
    lattice_tflops = nn_flop / (lattice_ms * 1e-3) / 1e12
    rate = float(lc.n_accepted.sum().cpu()) / (cycles * chains)
    lc.batch.check()

    def stats(trace, ms, sweeps):
        E = trace[:, :, 0] / N
        am = np.abs(trace[:, :, 1]) / N
        t_m, dt_m, _ = tau_int(am)
        t_e, dt_e, _ = tau_int(E)
        sweeps_per_s = sweeps / (ms * 1e-3)
        return {
            "tau_int_absm_sweeps": round(t_m, 2), "tau_int_absm_err": round(dt_m, 2),
            "tau_int_E_sweeps": round(t_e, 2), "tau_int_E_err": round(dt_e, 2),
            "ms_per_sweep_all_chains": round(ms / sweeps, 5),
            "samples_per_s_absm": round(chains * sweeps_per_s / (2 * t_m), 1),
            "samples_per_s_E": round(chains * sweeps_per_s / (2 * t_e), 1),
            "e_mean": binned_mean(E), "absm_mean": binned_mean(am),
        }

    sp = stats(trp, plain_ms, T)
    sl = stats(trl, learn_ms, cycles * k)
    # the same chains driven by the untrained network: what training gains
    net0 = lib.Net(L, max(batch, chains), params=nn_initial_params(7))
    lc0 = LearnedChains(net0, L, [beta] * chains, seed=301, sweeps_per_proposal=k)
    for _ in range(100):
        lc0.cycle()
    lc0.n_accepted.zero_()
    tr = torch.empty((cycles * k, chains, 2), dtype=torch.int64, device=dev)

    def run_cycles0():
        for c in range(cycles):
            lc0.cycle(trace=tr[c * k:(c + 1) * k])

    _, learn0_ms = timed(run_cycles0)
    s0 = stats(tr.cpu().numpy(), learn0_ms, cycles * k)
    rate0 = float(lc0.n_accepted.sum().cpu()) / (cycles * chains)
    lc0.batch.check()
    del tr, lc0, net0
    # cost model: a cycle of k sweeps decorrelates |m| by about k / (2 tau)
    # independent samples per chain, an accepted proposal by one more; the
    # learned chain beats the plain one when a > (k / (2 tau)) (T_prop / T_k)
    t_k = plain_ms / T * k
    t_prop = learn_ms / cycles - t_k
    per_cycle = k / (2 * sp["tau_int_absm_sweeps"])
    cost_model = {
        "sweeps_ms_per_cycle": round(t_k, 4), "proposal_ms_per_cycle": round(t_prop, 4),
        "plain_samples_per_cycle": round(per_cycle, 4),
        "acceptance_needed": round(per_cycle * t_prop / t_k, 3),
        "proposal_ms_needed_at_this_acceptance": round(rate * t_k / per_cycle, 5),
        "proposal_ms_needed_at_full_acceptance": round(t_k / per_cycle, 4),
    }
    train_gbs = steps * batch * N * NN_TRAIN_BYTES_PER_SITE / (train_ms * 1e-3) / 1e9
    rec = {
        "metric": METRIC,
        "value": sl["samples_per_s_absm"],
        "unit": "independent samples/s (|m|, tau_int-normalised)",
        "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(learn_ms / cycles, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 weights / fp32 accumulate; u32 sweeps", "data": "synthetic",
        "config": {
            "workload": f"2D Ising L={L}, beta={beta}, {chains} chains; masked-conv autoregressive "
                        f"proposal (4 layers, 16 channels, 3x3) trained on "
                        f"{snaps * chains} plain-sampler configurations; one Z2-symmetrised "
                        f"whole-lattice proposal per {k} sweeps",
            "L": L, "beta": beta, "chains": chains, "train_configs": snaps * chains,
            "train_steps": steps, "parallelism": "single GPU",
        },
        "learned": sl, "plain": sp,
        "learned_over_plain": {
            "absm": round(sl["samples_per_s_absm"] / sp["samples_per_s_absm"], 4),
            "E": round(sl["samples_per_s_E"] / sp["samples_per_s_E"], 4),
        },
        "acceptance_rate": round(rate, 5),
        "untrained": dict(s0, acceptance_rate=round(rate0, 5)),
        "trained_over_untrained": {
            "acceptance": round(rate / max(rate0, 1e-12), 1) if rate0 > 0 else None,
            "samples_per_s_absm": round(sl["samples_per_s_absm"] / s0["samples_per_s_absm"], 4),
        },
        "cost_model": cost_model,
        "training": {"ms": round(train_ms, 1), "steps": steps, "batch": batch,
                     "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
                     "data_generation_ms": round(gen_ms, 1)},
        "roofline": {
            "bound": "mfma",
            "achieved": round(wave_tflops, 3), "peak": BF16_MATRIX_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(wave_tflops / BF16_MATRIX_PEAK_TFLOPS, 4), "traffic": None,
            "kernel": "k_nn_wave (sampling: the proposals and their log q_sym, "
                      "2 waves per configuration)",
            "kernel_ms": round(wave_ms, 4),
            "work": f"{chains} configurations x 2 signs x {N} sites x "
                    f"({NN_WAVE_BF16_MAC_PER_SITE} bfloat16 + {NN_WAVE_F32_MAC_PER_SITE} "
                    "float32 multiply-adds)",
            "note": f"{3 * L - 2} dependent anti-diagonal steps per configuration: the kernel "
                    "is bound by the latency of a step, not by the matrix cores' rate",
        },
        "logq_roofline": {
            "bound": "mfma",
            "achieved": round(lattice_tflops, 3), "peak": BF16_MATRIX_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(lattice_tflops / BF16_MATRIX_PEAK_TFLOPS, 4),
            "traffic": None,
            "kernel": "k_nn_lattice (log q_sym of the current states, a layer at a time over "
                      "the whole lattice in LDS)",
            "kernel_ms": round(lattice_ms, 4),
            "work": "as roofline",
        },
        "training_roofline": {
            "bound": "hbm",
            "achieved": round(train_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(train_gbs / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "training step (forward, backward, one reduction, Adam)",
            "work": f"{NN_TRAIN_BYTES_PER_SITE} bytes per site per configuration",
        },
    }
    print(json.dumps(rec), flush=True)


def cpu_baseline_ea(J, betas, seed: int, every: int, target_s: float, draws: str = "plane"):
    """The oracle on a bounded sample of the spin-glass workload: all
    replicas from the same random starts, the first sweeps."""
    import oracle

    mode = oracle.MODE_PLANE if draws == "plane" else oracle.MODE_SITE
    threads = max(1, min(16, os.cpu_count() or 1))
    R, L = len(betas), J.shape[1]
    spins = np.stack([oracle.ea_init(L, oracle.START_RANDOM, seed, r) for r in range(R)])
    E = np.array([oracle.ea_energy(x, J) for x in spins])
    perm = np.arange(R, dtype=np.int32)
    t0 = time.perf_counter()
    oracle.ea_run(spins, J, betas, seed, 0, 1, every, perm, E, trace=False, nthreads=threads,
                  mode=mode)
    one = time.perf_counter() - t0
    n = max(1, min(50, int(target_s / max(one, 1e-6))))
    t0 = time.perf_counter()
    oracle.ea_run(spins, J, betas, seed, 1, n, every, perm, E, trace=False, nthreads=threads,
                  mode=mode)
    dt = time.perf_counter() - t0
    return {"value": R * L ** 3 * n / (dt * 1e9), "unit": "spin-flip attempts/ns", "cores": threads,
            "kind": "oracle",
            "sample": f"all {R} replicas, sweeps 1..{n} ({dt:.1f} s), exchange every {every}, "
                      f"{draws} draws"}


def bench_ea(args):
    import torch

    import paper_2402_06415_amd as lib
    from paper_2402_06415_amd.workloads import ea_bonds, ea_workload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = ea_workload()
    L, betas, every = wl["L"], wl["beta"], wl["every"]
    R = len(betas)
    nsw = args.sweeps if args.sweeps != 1000 else wl["sweeps"]
    J = ea_bonds(L, wl["bond_seed"])
    plane = args.draws == "plane"
    kernel = "k_ea_halfsweep_bit" if plane else "k_ea_halfsweep"
    g = lib.SpinGlass(J, betas, seed=wl["seed"], device=dev, draws=args.draws)
    # one block of sweeps (4 launches per sweep; ten exchange periods, so that
    # the plane mode's packing and unpacking at the ends of a call are
    # amortised) captured once and replayed
    block = every * 10 if nsw % (every * 10) == 0 else every
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        g.sweep(block, every)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g.sweep(block, every)
    stream = torch.cuda.current_stream()
    reps = nsw // block

    def step():
        g.init("random")
        for _ in range(reps):
            graph.replay()
        return g.measure()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    g.check()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    sw = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for k in range(args.steps):
        g.init("random")
        if k == args.steps - 1:
            sw[0].record(stream)
        for _ in range(reps):
            graph.replay()
        if k == args.steps - 1:
            sw[1].record(stream)
        g.measure()
    ev[1].record(stream)
    torch.cuda.synchronize()
    total_ms = ev[0].elapsed_time(ev[1])
    sweep_ms = sw[0].elapsed_time(sw[1])
    blocks = g.rng_blocks()
    t, perm, E, acc = g.state()
    g.check()
    attempts = R * L ** 3 * nsw
    ms_per_step = total_ms / args.steps
    achieved_tops = blocks * PHILOX_OPS_PER_BLOCK / (sweep_ms * 1e-3) / 1e12
    prof = profiled_traffic(kernel, "ea_plane_L128_R64" if plane else "ea_L128_R64",
                            "ea_kernels.hip") if (L == 128 and R == 64) else None
    eff_gbs = attempts * 2.0 / (sweep_ms * 1e-3) / 1e9
    rec = {
        "metric": METRIC,
        "value": round(attempts / (ms_per_step * 1e6), 3),
        "unit": "spin-flip attempts/ns",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {
            "workload": f"3D Edwards-Anderson +-J glass L={L} (bonds seed {wl['bond_seed']}), {R} "
                        f"replicas at beta in [0.5, 1.2], exchange every {every} sweeps, {nsw} "
                        "sweeps per step (HIP-graph replays of ten exchange periods) + init + recount",
            "L": L, "replicas": R, "sweeps_per_step": nsw, "every": every,
            "draws": args.draws,
            "layout": "int8 in HBM, colour bit planes in the workspace during a call" if plane
                      else "int8", "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "alu", "achieved": round(achieved_tops, 3), "peak": round(VALU_PEAK_TOPS, 2),
            "unit": "TOP/s", "frac": round(achieved_tops / VALU_PEAK_TOPS, 4),
            "traffic": round(prof["hbm_read_bytes_per_launch"] + prof["hbm_write_bytes_per_launch"])
            if prof else None,
            "traffic_unit": f"bytes per {kernel} launch (rocprofv3, copy-scaled)",
            "kernel": f"{kernel} (+ reduce and exchange kernels)",
            "kernel_ms": round(sweep_ms, 3),
            "work": f"{blocks} Philox4x32-10 blocks x {PHILOX_OPS_PER_BLOCK} int ops in the last step",
        },
        "hbm_roofline": {"achieved": round(eff_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(eff_gbs / HBM_PEAK_GBS, 4),
                         "note": "algorithmic 2 B/attempt (INT8 spins read + written per sweep); "
                                 "128 MiB of spins + 6 MiB of bonds"},
        "swap_acceptance": [round(float(a) / (nsw // every / 2), 4) for a in acc],
        "sweep_index": t,
    }
    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        c = torch.empty_like(a)
        c.copy_(a)
        torch.cuda.synchronize()
        rec["copy_calibration_bytes"] = 1 << 30
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline_ea(J, betas, wl["seed"], every, args.cpu_seconds,
                                              args.draws)
    print(json.dumps(rec), flush=True)


# the paper's own XY timing: 42.36 us per MC step at L = 32 (float64, FPGA)
PAPER_XY_L32_US = 42.36


def bench_xy(args):
    """Time per Monte Carlo step and internal energy U = <H>/L^2 of the XY
    model at T = 0.85 for L = 8..128, ten independent lattices per size."""
    import torch

    import paper_2402_06415_amd as lib
    from paper_2402_06415_amd.analysis import binned_mean

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    beta, seeds, steps = 1.0 / 0.85, 10, (args.sweeps if args.sweeps != 1000 else 10_000)
    stream = torch.cuda.current_stream()
    sizes = {}
    for L in (8, 16, 32, 64, 128):
        g = lib.XYLattices(L, seeds, seed=1 + L, start="random", device=dev)
        g.sweep(beta, max(steps // 5, 1), trace=False)  # equilibration
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        E = g.sweep(beta, steps)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        g.check()
        U, dU = binned_mean(E.cpu().numpy() / (L * L))
        _, acc = g.state()
        sizes[str(L)] = {"us_per_step": round(ms * 1e3 / steps, 3),
                         "attempts_per_ns_10_lattices": round(seeds * L * L * steps / (ms * 1e6), 4),
                         "U": round(U, 6), "U_err": round(dU, 6),
                         "acceptance": round(float(acc.sum()) / (seeds * L * L * (steps + steps // 5)), 4)}
    l32 = sizes["32"]
    value = 1024 / (l32["us_per_step"] * 1e3)  # attempts/ns of one L = 32 lattice
    rec = {
        "metric": METRIC, "value": round(value, 4), "unit": "spin-flip attempts/ns",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": round(l32["us_per_step"] / 1e3, 6),
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": round(PAPER_XY_L32_US / l32["us_per_step"], 3),
        "vs_baseline_note": "paper's FPGA: 42.36 us per MC step at L=32, float64 (its own hardware)",
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"2D XY model, T=0.85, random starts, {steps} MC steps per size, "
                               f"{seeds} independent lattices per size (value: one L=32 lattice)",
                   "sizes": [8, 16, 32, 64, 128], "parallelism": "single GPU"},
        "sizes": sizes,
    }
    if not args.no_cpu_baseline:
        import oracle

        th = oracle.xy_init(32, oracle.START_RANDOM, 33, 0)
        n = 200
        t0 = time.perf_counter()
        oracle.xy_sweep(th, 33, 0, 0, n, beta)
        dt = time.perf_counter() - t0
        rec["cpu_baseline"] = {"value": 1024 * n / (dt * 1e9), "unit": "spin-flip attempts/ns",
                               "cores": 1, "kind": "oracle",
                               "sample": f"one L=32 lattice, {n} MC steps ({dt:.2f} s), "
                                         f"{dt / n * 1e6:.1f} us per step"}
    print(json.dumps(rec), flush=True)


def bench_scaling(args):
    """Time per sweep against the number of sites N = L^2 for both layouts,
    the paper's scaling study (L = 8..128) extended to large sides: t = aN + b
    fitted by least squares on relative residuals, and b/a, the lattice size
    at which the fixed cost of a sweep equals its cost per site."""
    import numpy as np
    import torch

    import paper_2402_06415_amd as lib

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    out = {}
    for layout, sides in (("int8", [8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096]),
                          ("bit1", [64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384])):
        rows = []
        for L in sides:
            n = int(min(10000, max(200, (1 << 30) // (L * L))))
            lat = lib.Lattice(L, layout, seed=args.seed, start="random", device=dev)
            lat.sweep(BETA, min(n, 50), record=False)
            stream = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            lat.sweep(BETA, n, record=False)
            e1.record(stream)
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / n
            lat.check()
            rows.append({"L": L, "sweeps": n, "us_per_sweep": round(us, 4),
                         "attempts_per_ns": round(L * L / (us * 1e3), 2)})
            print(f"[scaling] {layout} L={L}: {us:.3f} us per sweep", file=sys.stderr, flush=True)
            del lat
        N = np.array([r["L"] ** 2 for r in rows], float)
        t = np.array([r["us_per_sweep"] for r in rows])
        a, b = np.polyfit(N, t, 1, w=1.0 / t)
        out[layout] = {"sides": rows, "a_ns_per_site": round(a * 1e3, 6), "b_us": round(b, 3),
                       "b_over_a_sites": round(b / a, 1)}
    rec = {
        "metric": "time per sweep against lattice size, t = aN + b",
        "value": out["bit1"]["a_ns_per_site"],
        "unit": "ns per site (bit-packed)",
        "n_gpus": 1, "steps": 1, "warmup": 1, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8 / u32", "data": "synthetic",
        "config": {"workload": "one 2D Ising lattice per side, random start seed "
                               f"{args.seed}, beta=0.4406868, int8 L=8..4096 and bit-packed "
                               "L=64..16384, sweeps in one call, no observables",
                   "parallelism": "single GPU"},
        "layouts": out,
    }
    print(json.dumps(rec), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "decomposition is a design, not a build.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "learned":
        return bench_learned(args)
    if args.workload == "ea":
        return bench_ea(args)
    if args.workload == "xy":
        return bench_xy(args)
    if args.workload == "scaling":
        return bench_scaling(args)
    import torch

    import paper_2402_06415_amd as lib

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    L, nsw = args.L, args.sweeps
    flags = lib.FLAG_GLOBAL_HALFSWEEP if args.global_halfsweep else 0
    layout = args.layout
    lat = lib.Lattice(L, layout, seed=args.seed, start="random", device=dev, flags=flags)
    stream = torch.cuda.current_stream()
    out = torch.zeros(2, dtype=torch.int64, device=dev)

    def step():
        lat.init("random")                    # random start, seed 7
        lat.sweep(BETA, nsw, record=False)    # thresholds on the host + persistent sweep kernel
        return lat.measure()                  # recount E and M

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    lat.check()

    # timed region: K steps between two events on the library's stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    sw_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
             for _ in range(args.steps)]
    blocks_before = None
    torch.cuda.synchronize()
    ev[0].record(stream)
    for k in range(args.steps):
        lat.init("random")
        sw_ev[k][0].record(stream)
        lat.sweep(BETA, nsw, record=False)
        sw_ev[k][1].record(stream)
        out = lat.measure()
    ev[1].record(stream)
    torch.cuda.synchronize()
    total_ms = ev[0].elapsed_time(ev[1])
    sweep_ms = sum(a.elapsed_time(b) for a, b in sw_ev) / args.steps
    lat.check()
    E, M = (int(v) for v in out.cpu().tolist())
    # Philox blocks of one step, outside the timed region: the same chain on a
    # lattice that counts its draws (the timed kernels do not count)
    counted = lib.Lattice(L, layout, seed=args.seed, start="random", device=dev,
                          flags=flags | lib.FLAG_COUNT_DRAWS)
    counted.sweep(BETA, nsw, record=False)
    blocks = counted.rng_blocks()
    assert tuple(int(v) for v in counted.measure().cpu().tolist()) == (E, M)
    del counted

    ms_per_step = total_ms / args.steps
    attempts = L * L * nsw
    value = attempts / (ms_per_step * 1e6)
    # roofline of the sweep kernel: integer VALU work of the Philox draws the
    # method consumed, against the chip's VALU lane-op peak
    achieved_tops = blocks * PHILOX_OPS_PER_BLOCK / (sweep_ms * 1e-3) / 1e12
    # effective HBM roofline: every spin read and written once per sweep,
    # 2 bits per attempt bit-packed, 2 bytes as int8
    per_attempt = 0.25 if layout == "bit1" else 2.0
    alg_bytes = attempts * per_attempt
    eff_gbs = alg_bytes / (sweep_ms * 1e-3) / 1e9
    if layout == "bit1":
        # the library's tile plan keeps the lattice in LDS while its tiles fit
        # (L <= 16384 on 256 CUs); larger lattices run one launch per
        # half-sweep from global memory
        kernel_name = "k_halfsweep_bit1" if args.global_halfsweep else bit1_sweep_kernel(
            L, torch.cuda.get_device_properties(0).multi_processor_count)
        tiles = kernel_name != "k_halfsweep_bit1"
    else:
        # int8: tiles of rows in LDS for 64 < L <= 4096 (L % 8 == 0), else
        # one resident workgroup up to L = 128, else a launch per half-sweep
        span = L % 8 == 0 and L * L < (1 << 31)  # the byte-parallel span kernel
        if args.global_halfsweep:
            kernel_name = "k_halfsweep_int8_quad" if span else "k_halfsweep_int8"
        elif 64 < L <= 4096 and L % 8 == 0:
            kernel_name = "k_sweep_int8_tiles"
        elif L <= 128:
            kernel_name = "k_sweep_int8_resident"
        else:
            kernel_name = "k_halfsweep_int8_quad" if span else "k_halfsweep_int8"
        tiles = kernel_name in ("k_sweep_int8_resident", "k_sweep_int8_tiles")
    prof = profiled_traffic(kernel_name) if (layout == "bit1" and L == 4096 and nsw == 1000) else None
    copy_gbs = measured_copy_gbs(torch, dev)
    traffic = (prof["hbm_read_bytes_per_launch"] + prof["hbm_write_bytes_per_launch"]) if prof else None
    valu_per_word, ceiling = valu_ceiling(prof, L * L // 32 * nsw) if layout == "bit1" else (None, None)
    rec = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "spin-flip attempts/ns",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32" if layout == "bit1" else "i8",
        "data": "synthetic",
        "config": {
            "workload": f"2D Ising L={L} " + ("one bit per spin" if layout == "bit1" else "int8")
                        + f", random start seed {args.seed}, "
                        f"beta={BETA}, {nsw} checkerboard sweeps + init + recount per step",
            "L": L, "sweeps_per_step": nsw, "beta": BETA, "seed": args.seed,
            "layout": layout, "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved_tops, 3),
            "peak": round(VALU_PEAK_TOPS, 2),
            "unit": "TOP/s",
            "frac": round(achieved_tops / VALU_PEAK_TOPS, 4),
            "traffic": round(traffic) if traffic else None,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "kernel": kernel_name,
            "kernel_ms": round(sweep_ms, 4),
            "work": f"{blocks} Philox4x32-10 blocks x {PHILOX_OPS_PER_BLOCK} int ops per launch "
                    "(the blocks the chain needs, counted on a same-chain lattice)",
            "valu_issue_utilisation": round(prof["valu_utilisation"], 3) if prof else None,
            "valu_per_word": round(valu_per_word, 1) if valu_per_word else None,
            "valu_ceiling_attempts_per_ns": round(ceiling, 1) if ceiling else None,
            "frac_of_valu_ceiling": round(value / ceiling, 4) if ceiling else None,
        },
        "hbm_roofline": {
            "achieved": round(eff_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(eff_gbs / HBM_PEAK_GBS, 4),
            "copy_measured": round(copy_gbs, 1),
            "frac_of_copy": round(eff_gbs / copy_gbs, 4),
            "note": f"algorithmic {per_attempt:g} B/attempt"
                    + ("; the lattice stays in LDS during a call" if tiles else "; lattice in HBM")
                    + "; copy_measured: a 1 GiB device copy on this GPU, read + write bytes",
        },
        "E_final": E, "M_final": M,
    }
    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        rec["copy_calibration_bytes"] = 1 << 30
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(L, args.seed, args.cpu_seconds, layout)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
