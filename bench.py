#!/usr/bin/env python3
"""Benchmark of the Floquet-period hot path on one MI355X.

Workload (one "step"): 10 Floquet periods of the L = 30 XYZ-plus-fields chain
(complex64 state, 8 GiB, plain fused FP32 sweep, T = 0.25, seed 2111) followed
by one energy-density readout, i.e. the record interval of that run.  Inputs
are synthetic and resident in HBM before timing starts.

Prints ONE JSON line.  Besides periods/s it reports:
  roofline      the dominant kernel (the fused sweep), timed live with HIP
                events on the launch stream over a sweep-only region
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same workload
  adjoint       the adjoint/forward time ratio of the gradient at L = 24
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Floquet periods/sec + HBM GB/s at L=30 fp32; adjoint/forward time ratio"
PEAK_HBM_GBPS = 8000.0
# MI355X's published FP32 vector peak (TFLOP/s): 256 CUs x 4 SIMD x 16 lanes
# x 2 FMA per lane and cycle x 2 flop x 2.4 GHz.  The roofline fraction is
# taken against it.  This build emits no packed FP32; the second FMA per cycle
# comes from issuing two waves' FMAs together, which gfx950 does for FMAs
# that read no scalar register (measured by the probes below).
PEAK_FP32_PUBLISHED = 157.3
# One FMA per lane and cycle: the ceiling of FMAs that read a scalar
# register (they do not issue in pairs).  Reported beside the published
# fraction.
PEAK_FP32_VALU = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


# HBM bytes per sweep launch from two rocprofv3 --pmc runs (FETCH_SIZE, then
# WRITE_SIZE) of "bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-adjoint
# --no-l34 --calibrate-copy", each scaled by what the counter reads for the
# plain 8 GiB device copy in the same run (FETCH_SIZE read 4.0 GiB -> x2;
# WRITE_SIZE read 8.0 GiB -> x1).  Valid only for the kernel code it was taken
# on: the key is a hash of kernels.hip and fl_common.h with comments and
# whitespace removed.
TRAFFIC = {"kernel_code_sha256_16": "2dfed1bd7b4b735a", "fetch_gib_raw": 4.0002, "fetch_scale": 2.0,
           "write_gib_raw": 8.0, "write_scale": 1.0}


def kernel_code_hash():
    import hashlib
    import re
    h = hashlib.sha256()
    for name in ("kernels.hip", "fl_common.h"):
        with open(os.path.join(ROOT, "paper_2111_08044_amd", "csrc", name)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(re.sub(r"\s+", " ", text).strip().encode())
    return h.hexdigest()[:16]


def measured_traffic():
    if kernel_code_hash() != TRAFFIC["kernel_code_sha256_16"]:
        return None
    gib = TRAFFIC["fetch_gib_raw"] * TRAFFIC["fetch_scale"] + TRAFFIC["write_gib_raw"] * TRAFFIC["write_scale"]
    return gib * 2**30


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--L", type=int, default=30)
    ap.add_argument("--periods-per-step", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-l34", action="store_true", help="skip the L=34 (128 GiB, in place) leg")
    ap.add_argument("--cpu-sample-gates", type=int, default=3)
    ap.add_argument("--study", choices=["precision", "echo", "gue", "long", "sizes", "adjoint"], default=None,
                    help="instead of the throughput benchmark: error versus depth of the precision "
                         "variants against an FP64 GPU run (precision), the echo overlap error (echo), "
                         "heating of the paper's GUE circuit versus drive frequency (gue), or the energy "
                         "density every 100 periods of a long run (long, with --L 34), time per "
                         "period and per readout versus L = 16..34 (sizes), or only the adjoint/forward "
                         "ratio at --L (adjoint: one forward and one gradient of 200 periods, K = 50, "
                         "after one untimed repetition)")
    ap.add_argument("--cpu-baseline-scaling", action="store_true",
                    help="only the cpu_baseline leg, at L = 20..28: the oracle's time per period and its "
                         "a L 2^L fit (no GPU)")
    ap.add_argument("--max-periods", type=int, default=10000)
    ap.add_argument("--variants", type=str, default="plain,dense6_fp32,dense6_bf16x3",
                    help="complex64 variants of --study precision")
    ap.add_argument("--omegas", type=str, default="5,5.5,6,6.5,7,7.5,8",
                    help="drive frequencies of --study gue")
    ap.add_argument("--tmax", type=float, default=2e5, help="longest time (units of 1/J) of --study gue")
    ap.add_argument("--echo-model", choices=["xyz", "gue"], default="xyz",
                    help="circuit of --study echo: the XYZ+fields chain or the paper's GUE circuit")
    ap.add_argument("--omega", type=float, default=8.0, help="drive frequency of --study echo --echo-model gue")
    ap.add_argument("--depths", type=str, default=None,
                    help="comma-separated echo depths t_f of --study echo (default: 1, 2, 5, 10, ... up to "
                         "--max-periods)")
    ap.add_argument("--sweep-only", type=int, default=0, metavar="N",
                    help="only initialise the state and run N periods of the plain sweep, then exit "
                         "(a short program for hardware counter runs)")
    ap.add_argument("--sweep-variant", choices=["plain", "dense6_fp32", "dense6_bf16x3", "dense4_fp32"],
                    default="plain", help="the complex64 variant --sweep-only and --study adjoint run")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also copy the state once (a plain device copy of known size, the reference "
                         "for scaling hardware byte counters)")
    return ap.parse_args()


def measured_ceilings(torch, psi):
    """Ceilings measured on the device: the FP32 FMA rates of two plain FMA
    loops (libflprobe.so, no packed FP32; coefficients in scalar registers,
    then in vector registers) and the bandwidth of a plain device copy of the
    state (read + write), each the best of several runs, timed with events on
    the current stream."""
    import ctypes
    out = {}
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    lib_path = os.path.join(ROOT, "paper_2111_08044_amd", "libflprobe.so")
    if os.path.exists(lib_path):
        probe = ctypes.CDLL(lib_path)
        blocks, iters = 256 * 32, 20000
        buf = torch.empty(blocks * 256, dtype=torch.float32, device=psi.device)
        for name, key in (("flp_fma_loop", "fma_loop_tflops"), ("flp_fma_loop_v", "fma_loop_vgpr_tflops")):
            f = getattr(probe, name)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
            best = 0.0
            for _ in range(4):
                ev0.record(stream)
                rc = f(buf.data_ptr(), blocks, iters, ctypes.c_void_p(stream.cuda_stream))
                ev1.record(stream)
                torch.cuda.synchronize()
                if rc != 0:
                    raise RuntimeError(f"{name} failed ({rc})")
                best = max(best, 2.0 * 16 * iters * blocks * 256 / (ev0.elapsed_time(ev1) / 1e3) / 1e12)
            out[key] = round(best, 2)
        del buf
    tmp = torch.empty_like(psi)
    best = 0.0
    for _ in range(3):
        ev0.record(stream)
        tmp.copy_(psi)
        ev1.record(stream)
        torch.cuda.synchronize()
        best = max(best, 2.0 * psi.numel() * psi.element_size() / (ev0.elapsed_time(ev1) / 1e3) / 1e9)
    out["copy_gbps"] = round(best, 1)
    del tmp
    return out


def plan_passes(fl, L, n):
    """Number of sweep launches the library runs for n periods (header word 3
    of the flattened plan)."""
    return int(fl.fl_plan_query(L, "c64", 0, n, False)[3])


DENSE = {  # plan kind, MFMA flop per amplitude per window, MFMA peak (TFLOP/s, dense)
    "dense6_fp32": (4, 512.0, 157.3),
    "dense6_bf16x3": (4, 1536.0, 2516.6),
    "dense4_fp32": (5, 128.0, 157.3),
}


def _dense_groups(fl, L, n, kind=4):
    """Register groups (= windows) of each pass of a dense plan for n periods."""
    words = [int(x) for x in fl.fl_plan_query(L, "c64", kind, n, False)]
    npasses, i, out = words[3], 4, []
    for _ in range(npasses):
        ng = words[i + 1]
        i += 3
        groups = []
        for _ in range(ng):
            nops = words[i + 1]
            groups.append(words[i])
            i += 2 + 3 * nops
        out.append(groups)
    return out


def cpu_baseline(L, nsample):
    """The oracle as it stands, timed on a bounded sample: nsample gate
    applications spread over the chain at full size L, scaled to periods/s."""
    import numpy as np

    import floquet_inputs as fin
    import oracle as O
    w = fin.xyz_workload(L)
    hs = O.xyz_bond_hamiltonians(L, w["J"], w["fields"])
    G = O.floquet_gates(hs, w["T"])
    psi = np.full(1 << L, 1.0 / np.sqrt(float(1 << L)), dtype=np.complex128)
    bonds = [int(round(x)) for x in np.linspace(0, L - 2, nsample)]
    t0 = time.perf_counter()
    for b in bonds:
        psi = O.apply_bond(psi, L, b, G[b])
    dt = time.perf_counter() - t0
    s_per_gate = dt / len(bonds)
    s_per_period = s_per_gate * (L - 1)
    return {"value": 1.0 / s_per_period, "unit": "periods/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(bonds)} FP64 gate applications (bonds {bonds}) at L={L}, "
                      f"{dt:.1f} s, scaled by {L - 1} gates/period; numpy einsum, single thread",
            "s_per_period": s_per_period, "host": cpu_model(), "host_cpus": os.cpu_count()}


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), else the machine type."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline_scaling(Ls, nrep=2):
    """The cpu_baseline leg at several chain lengths: wall time of one full
    period of the oracle (FP64, one gate at a time), fitted to a L 2^L (the
    cost the paper states, Sec. V), and the fit's value at L = 30 beside the
    direct L = 30 sample of cpu_baseline."""
    import numpy as np

    import floquet_inputs as fin
    import oracle as O
    rows = []
    for L in Ls:
        w = fin.xyz_workload(L)
        hs = O.xyz_bond_hamiltonians(L, w["J"], w["fields"])
        G = O.floquet_gates(hs, w["T"])
        psi0 = O.product_state(w["spinors"])
        best = float("inf")
        for _ in range(nrep if L < 28 else 1):
            t0 = time.perf_counter()
            O.evolve(psi0, L, G, 1)
            best = min(best, time.perf_counter() - t0)
        rows.append({"L": L, "s_per_period": round(best, 4), "ns_per_amp_gate": round(1e9 * best / ((L - 1) * 2.0**L), 3)})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    x = np.array([r["L"] * 2.0**r["L"] for r in rows])
    t = np.array([r["s_per_period"] for r in rows])
    a = float(np.dot(t, x) / np.dot(x, x))
    return {"cpu_baseline_scaling": "oracle", "fit": "t = a L 2^L", "a_ns": round(a * 1e9, 4),
            "fit_s_per_period_L30": round(a * 30 * 2.0**30, 2), "rows": rows, "cores": 1,
            "host": cpu_model(), "host_cpus": os.cpu_count()}


def adjoint_ratio(fl, torch, L=24, n=200, K=50, variant="plain"):
    import floquet_inputs as fin
    w = fin.xyz_workload(L)
    eng = fl.FloquetEngine(L, "c64", variant)
    eng.set_xyz(w["J"], w["fields"], w["T"])
    psi = eng.new_state()
    gens = fl.fl_xyz_generators(L)
    lam = torch.empty_like(psi)
    ck = [torch.empty_like(psi) for _ in range(n // K)]
    res = {}
    for rep in range(2):          # first repetition warms up plans and caches
        eng.init(psi, w["spinors"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(n // K):
            ck[s].copy_(psi)
            eng.step(psi, K)
        E, _ = eng.energy(psi)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g = fl.fl_grad(eng.ctx, psi, ck, n, K, gens, lam)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res = {"L": L, "variant": variant, "n_periods": n, "ckpt_every": K, "forward_s": t1 - t0,
               "backward_s": t2 - t1,
               "ratio_backward_over_forward": (t2 - t1) / (t1 - t0),
               "ratio_total_over_forward": (t2 - t0) / (t1 - t0), "dE_dT": float(g[-1])}
    return res


def _depths(nmax):
    d, out = 1, []
    while d <= nmax:
        for m in (1, 2, 5):
            if m * d <= nmax:
                out.append(m * d)
        d *= 10
    return out


def precision_study(fl, torch, L, nmax, variants=("plain", "dense6_fp32", "dense6_bf16x3")):
    """Infidelity 1 - |<psi64|psi>|^2/(|psi64|^2 |psi|^2), energy-density error
    |e - e64| and norm drift of the complex64 variants (plain FP32 sweep, FP32
    MFMA windows, split-BF16x3 MFMA windows) against an FP64 GPU run, at
    depths 1, 2, 5, 10, ... up to nmax periods (same gates, same start)."""
    import floquet_inputs as fin
    w = fin.xyz_workload(L)
    h = fl.fl_xyz_bonds(L, w["J"], w["fields"])
    ref = fl.FloquetEngine(L, "c128")
    ref.set_bonds(h, w["T"])
    p64 = ref.new_state()
    ref.init(p64, w["spinors"])
    engines, states = {}, {}
    for var in variants:
        e = fl.FloquetEngine(L, "c64", var)
        e.set_bonds(h, w["T"])
        engines[var] = e
        states[var] = e.new_state()
        e.init(states[var], w["spinors"])
    rows, t, times = [], 0, {k: 0.0 for k in ["c128"] + list(engines)}
    chunk = 500
    for d in _depths(nmax):
        while t < d:
            k = min(chunk, d - t)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ref.step(p64, k)
            torch.cuda.synchronize()
            times["c128"] += time.perf_counter() - t0
            for var, e in engines.items():
                t0 = time.perf_counter()
                e.step(states[var], k)
                torch.cuda.synchronize()
                times[var] += time.perf_counter() - t0
            t += k
            if t < d:
                print(json.dumps({"periods_done": t}), file=sys.stderr, flush=True)
        E64, N64 = ref.energy(p64)
        row = {"period": d, "e64": E64 / (L * N64), "norm64_minus_1": N64 - 1.0}
        for var, e in engines.items():
            ov, n64, n = ref.overlap(p64, states[var])
            E, N = e.energy(states[var])
            row[var] = {"infidelity": 1.0 - abs(ov) ** 2 / (n64 * n), "abs_e_err": abs(E / (L * N) - E64 / (L * N64)),
                        "overlap_error": abs(1.0 - ov), "norm_minus_1": N - 1.0}
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    return {"study": "precision", "L": L, "periods": t, "rows": rows,
            "ms_per_period": {k: round(v / t * 1e3, 3) for k, v in times.items()}}


def echo_study(fl, torch, L, nmax, model="xyz", omega=8.0, depths=None):
    """Echo of Sec. V: evolve d periods with U_F, then d with U_F^dagger, and
    report |1 - <psi0|psi'0>| and the infidelity, complex64 plain sweep.
    model "xyz": the XYZ+fields chain from a product state; "gue": the paper's
    GUE circuit at drive frequency omega from the ground state of H_o (the
    paper's own echo setting, Sec. V)."""
    import floquet_inputs as fin
    e = fl.FloquetEngine(L, "c64")
    psi0, psi = e.new_state(), e.new_state()
    if model == "gue":
        e.set_paper_model(fin.gue_bond_sample(L), omega)
        e.init_ground_pairs(psi0)
    else:
        w = fin.xyz_workload(L)
        e.set_xyz(w["J"], w["fields"], w["T"])
        e.init(psi0, w["spinors"])
    rows = []
    chunk = 1000 if L < 32 else 100   # a progress line every ~25 s at L = 34
    t_start = time.perf_counter()
    for d in (depths or _depths(nmax)):
        psi.copy_(psi0)
        for dagger in (False, True):
            left = d
            while left > 0:   # chunks, so that a long run reports its progress
                k = min(left, chunk)
                e.step(psi, k, dagger=dagger)
                left -= k
                if d > chunk:
                    torch.cuda.synchronize()
                    print(json.dumps({"t_f_periods": d, "dagger": dagger, "left": left,
                                      "elapsed_s": round(time.perf_counter() - t_start, 1)}), file=sys.stderr, flush=True)
        ov, n0, n1 = e.overlap(psi0, psi)
        row = {"t_f_periods": d, "overlap_error": abs(1.0 - ov), "infidelity": 1.0 - abs(ov) ** 2 / (n0 * n1),
               "norm_minus_1": n1 - 1.0}
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    return {"study": "echo", "L": L, "model": model, "omega": omega if model == "gue" else None, "rows": rows}


def gue_study(fl, torch, L, omegas, tmax, nrec=240):
    """The paper's own model (Sec. III A, IV): GUE bond terms H_k (one seeded
    sample), gates exp(-i H_k T) with T = 2 pi / omega, the ground state of H_o
    as the initial state; E(t) and sigma_E(t) of H-bar = sum_k H_k on
    log-spaced periods, and the heating rate Gamma = 1/(t2 - t1) with
    E(t_k) = E(0) exp(-k).  complex64 plain sweep.  A run stops once E/E(0)
    falls below exp(-2.5) or t reaches tmax."""
    import numpy as np

    import floquet_inputs as fin
    Hk = fin.gue_bond_sample(L)
    eng = fl.FloquetEngine(L, "c64")
    psi, ws = eng.new_state(), eng.new_state()
    out = []
    for om in omegas:
        T = 2.0 * np.pi / om
        eng.set_paper_model(Hk, om)
        eng.init_ground_pairs(psi)
        nmax = int(np.ceil(tmax / T))
        recs = np.unique(np.round(np.logspace(0, np.log10(nmax), nrec)).astype(np.int64))
        t_s, E_s, S_s = [], [], []

        def record(n):
            sig, e, _ = eng.energy_spread(psi, ws)   # of H0 = 2 H-bar
            t_s.append(n * T)
            E_s.append(0.5 * e)
            S_s.append(0.5 * sig)

        record(0)
        n, t0 = 0, time.perf_counter()
        t_said = t0
        for r in recs:
            eng.step(psi, int(r - n))
            n = int(r)
            record(n)
            if time.perf_counter() - t_said > 20.0:   # long runs report their progress
                print(json.dumps({"omega": om, "period": n, "E_over_E0": round(E_s[-1] / E_s[0], 6)}),
                      file=sys.stderr, flush=True)
                t_said = time.perf_counter()
            if E_s[-1] / E_s[0] < np.exp(-2.5):
                break
        torch.cuda.synchronize()
        G, t1, t2 = fl.thermalization_rate(t_s, E_s)
        row = {"omega": om, "T": T, "periods": n, "t_end": n * T, "seconds": round(time.perf_counter() - t0, 2),
               "E0": E_s[0], "sigma0": S_s[0], "E_end": E_s[-1], "sigma_end": S_s[-1],
               "gamma": G, "t1": t1, "t2": t2,
               "series": {"t": [round(x, 4) for x in t_s], "E_over_E0": [round(x / E_s[0], 6) for x in E_s],
                          "sigma": [round(x, 6) for x in S_s]}}
        print(json.dumps({k: v for k, v in row.items() if k != "series"}), file=sys.stderr, flush=True)
        out.append(row)
    def fit_over(rows):
        rows = [r for r in rows if r["gamma"] is not None]
        if len(rows) < 2:
            return None
        a, b = fl.fit_exponential_rate([r["omega"] for r in rows], [r["gamma"] for r in rows])
        return {"a": a, "b": b, "omegas": [r["omega"] for r in rows]}

    # the paper's fit leaves out the two lowest frequencies (early heating)
    fit = {"all": fit_over(out), "without_two_lowest": fit_over(sorted(out, key=lambda r: r["omega"])[2:])}
    # infinite-temperature spread: tr(H-bar^2) / 2^L = sum_k |H_k|_F^2 / 4
    # + 2 sum_k tr(R_k L_{k+1}) / 8 (R_k, L_k: H_k traced over its left / right
    # site; terms further apart vanish because every H_k is traceless)
    R4 = [np.einsum("aiaj->ij", H.reshape(2, 2, 2, 2)) for H in Hk]
    L4 = [np.einsum("iaja->ij", H.reshape(2, 2, 2, 2)) for H in Hk]
    var = np.sum(np.abs(Hk) ** 2) / 4.0 + 2.0 * sum(np.trace(R4[k] @ L4[k + 1]).real for k in range(L - 2)) / 8.0
    return {"study": "gue", "L": L, "seed": fin.DEFAULT_SEED, "tmax": tmax,
            "sigma_inf": float(np.sqrt(var)), "fit": fit, "rows": out}


def long_run(fl, torch, L, nmax, every=100):
    """The long run of the paper's largest single-device size (Sec. IV): the
    XYZ+fields chain at L (complex64, in place), the energy density every
    `every` periods up to nmax periods; periods/s of the whole run."""
    import floquet_inputs as fin
    w = fin.xyz_workload(L)
    eng = fl.FloquetEngine(L, "c64")
    eng.set_xyz(w["J"], w["fields"], w["T"])
    psi = eng.new_state()
    eng.init(psi, w["spinors"])
    E, N = eng.energy(psi)
    rows = [{"period": 0, "e": E / (L * N), "norm_minus_1": N - 1.0}]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = 0
    while n < nmax:
        k = min(every, nmax - n)
        eng.step(psi, k)
        n += k
        E, N = eng.energy(psi)
        rows.append({"period": n, "e": E / (L * N), "norm_minus_1": N - 1.0,
                     "elapsed_s": round(time.perf_counter() - t0, 2)})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    return {"study": "long", "L": L, "periods": n, "every": every, "wall_s": round(wall, 2),
            "periods_per_s": round(n / wall, 3), "rows": rows}


def size_scaling(fl, torch, Ls):
    """Time per period of the plain complex64 sweep and of one energy readout
    versus chain length (the cost the paper states grows as L 2^L, Sec. V):
    16 periods after 16 warm-up periods per size, HIP events on the launch
    stream."""
    import floquet_inputs as fin
    rows = []
    for L in Ls:
        w = fin.xyz_workload(L)
        eng = fl.FloquetEngine(L, "c64")
        eng.set_xyz(w["J"], w["fields"], w["T"])
        psi = eng.new_state()
        eng.init(psi, w["spinors"])
        eng.step(psi, 16)
        ev0, ev1, ev2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        stream = torch.cuda.current_stream()
        ev0.record(stream)
        eng.step(psi, 16)
        ev1.record(stream)
        e = eng.energy_density(psi)
        ev2.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / 16
        npass = plan_passes(fl, L, 16) / 16
        rows.append({"L": L, "ms_per_period": round(ms, 4), "periods_per_s": round(1e3 / ms, 2),
                     "passes_per_period": npass, "sweep_tflops": round(32.0 * (L - 1) * (1 << L) / (ms / 1e3) / 1e12, 2),
                     "ms_energy_readout": round(ev1.elapsed_time(ev2), 3), "energy_density_32": e})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
        del psi, eng
        torch.cuda.empty_cache()
    return {"study": "sizes", "rows": rows}


def l34_leg(fl, torch, periods=16):
    """L = 34 complex64 (128 GiB) in place: periods/s of the plain sweep and
    the energy density after the run."""
    import floquet_inputs as fin
    L = 34
    w = fin.xyz_workload(L)
    eng = fl.FloquetEngine(L, "c64")
    eng.set_xyz(w["J"], w["fields"], w["T"])
    psi = eng.new_state()
    eng.init(psi, w["spinors"])
    e0 = eng.energy_density(psi)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    ev0.record(stream)
    eng.step(psi, periods)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / periods
    t0 = time.perf_counter()
    e1 = eng.energy_density(psi)
    t_e = time.perf_counter() - t0
    npass = plan_passes(fl, L, 16) / 16
    res = {"L": L, "state_gib": (1 << L) * 8 / 2**30, "periods": periods, "ms_per_period": round(ms, 2),
           "periods_per_s": round(1e3 / ms, 3), "passes_per_period": npass,
           "hbm_gbps": round(16.0 * (1 << L) * npass / (ms / 1e3) / 1e9, 1),
           "sweep_tflops": round(32.0 * (L - 1) * (1 << L) / (ms / 1e3) / 1e12, 2),
           "energy_readout_s": round(t_e, 3), "energy_density_0": e0, "energy_density_end": e1}
    del psi, eng
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this engine has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    if args.cpu_baseline_scaling:
        print(json.dumps(cpu_baseline_scaling([20, 22, 24, 26, 28])), flush=True)
        return
    import numpy as np
    import torch

    import floquet_inputs as fin
    import paper_2111_08044_amd as fl

    L, m = args.L, args.periods_per_step
    torch.cuda.set_device(0)
    if args.study == "precision":
        print(json.dumps(precision_study(fl, torch, L, args.max_periods, args.variants.split(","))), flush=True)
        return
    if args.study == "echo":
        depths = [int(x) for x in args.depths.split(",")] if args.depths else None
        print(json.dumps(echo_study(fl, torch, L, args.max_periods, args.echo_model, args.omega, depths)), flush=True)
        return
    if args.study == "sizes":
        print(json.dumps(size_scaling(fl, torch, list(range(16, 35, 2)))), flush=True)
        return
    if args.study == "adjoint":
        print(json.dumps(adjoint_ratio(fl, torch, L=L, variant=args.sweep_variant)), flush=True)
        return
    if args.study == "long":
        print(json.dumps(long_run(fl, torch, L, args.max_periods)), flush=True)
        return
    if args.study == "gue":
        omegas = [float(x) for x in args.omegas.split(",")]
        print(json.dumps(gue_study(fl, torch, L, omegas, args.tmax)), flush=True)
        return
    w = fin.xyz_workload(L)
    eng = fl.FloquetEngine(L, "c64", args.sweep_variant if args.sweep_only > 0 else "plain")
    eng.set_xyz(w["J"], w["fields"], w["T"])
    psi = eng.new_state()
    eng.init(psi, w["spinors"])
    if args.sweep_only > 0:
        eng.step(psi, args.sweep_only)
        torch.cuda.synchronize()
        kind = {"plain": 0, "dense6_fp32": 4, "dense6_bf16x3": 4, "dense4_fp32": 5}[args.sweep_variant]
        print(json.dumps({"sweep_only": args.sweep_only, "L": L, "variant": args.sweep_variant,
                          "launches": int(fl.fl_plan_query(L, "c64", kind, args.sweep_only, False)[3])}), flush=True)
        return
    if args.calibrate_copy:
        tmp = torch.empty_like(psi)
        tmp.copy_(psi)
        torch.cuda.synchronize()
        del tmp
    e_series = []
    for _ in range(args.warmup):
        eng.step(psi, m)
        e_series.append(eng.energy_density(psi))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        eng.step(psi, m)
        e_series.append(eng.energy_density(psi))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    periods = args.steps * m
    periods_per_s = periods / wall

    step_passes = plan_passes(fl, L, m)
    readout_passes = int(fl.fl_plan_query(L, "c64", 6 if L > 13 else 2, 1, False)[3])
    # ---- the energy readout alone (fl_expect_energy synchronises; best of five)
    readout_ms = float("inf")
    for _ in range(5):
        t_r = time.perf_counter()
        eng.energy(psi)
        readout_ms = min(readout_ms, (time.perf_counter() - t_r) * 1e3)
    readout_ms = round(readout_ms, 3)

    # ---- dominant kernel: sweep-only region timed with events on the launch stream
    nblk = 16
    reps = 4
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    eng.step(psi, nblk)
    ev0.record(stream)
    for _ in range(reps):
        eng.step(psi, nblk)
    ev1.record(stream)
    torch.cuda.synchronize()
    sweep_ms = ev0.elapsed_time(ev1)
    launches = plan_passes(fl, L, nblk) * reps
    avg_launch_s = sweep_ms / 1e3 / launches
    gates = (L - 1) * nblk * reps
    flops = 32.0 * (1 << L) * gates                 # 16 FMA per amplitude per gate
    bytes_ = 16.0 * (1 << L) * launches             # read + write of every amplitude per pass
    achieved_tflops = flops / (sweep_ms / 1e3) / 1e12
    achieved_gbps = bytes_ / (sweep_ms / 1e3) / 1e9
    roof = {"kernel": "k_sweep_tiles<float,4,13,512,4,true>", "bound": "alu", "achieved": round(achieved_tflops, 3),
            "peak": PEAK_FP32_PUBLISHED, "unit": "TFLOP/s", "frac": round(achieved_tflops / PEAK_FP32_PUBLISHED, 4),
            "traffic": measured_traffic(), "avg_launch_ms": round(avg_launch_s * 1e3, 4),
            "flops_per_launch": flops / launches, "bytes_per_launch": bytes_ / launches,
            "peak_single_issue_fp32": round(PEAK_FP32_VALU, 2),
            "peak_single_issue_fp32_derivation": "256 CU x 4 SIMD x 16 lanes x 1 FMA x 2 flop x 2.4 GHz "
                                                  "(FMAs that read a scalar register)",
            "hbm_gbps": round(achieved_gbps, 1), "hbm_frac": round(achieved_gbps / PEAK_HBM_GBPS, 4),
            "passes_per_period": launches / (nblk * reps), "gates_per_pass": gates / launches}
    ceil = measured_ceilings(torch, psi)
    if "fma_loop_tflops" in ceil:
        roof["measured_fma_loop_sgpr_tflops"] = ceil["fma_loop_tflops"]
        roof["measured_fma_loop_vgpr_tflops"] = ceil["fma_loop_vgpr_tflops"]
        roof["frac_of_measured_fma_loop_vgpr"] = round(achieved_tflops / ceil["fma_loop_vgpr_tflops"], 4)
    roof["measured_copy_gbps"] = ceil["copy_gbps"]
    roof["hbm_frac_of_measured_copy"] = round(achieved_gbps / ceil["copy_gbps"], 4)

    out = {
        "metric": METRIC, "value": round(periods_per_s, 3), "unit": "periods/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"Floquet brickwork, L={L} XYZ+fields chain, complex64 state, plain fused sweep, "
                               f"T=0.25, seed 2111, {m} periods + 1 energy readout per step",
                   "L": L, "periods_per_step": m, "state_gib": (1 << L) * 8 / 2**30},
        "gates_per_s": round(periods_per_s * (L - 1), 1),
        # the step's own plan: plan_passes(m) sweep launches per m periods, plus one read of the state per readout pass
        "step_sweep_passes": step_passes,
        "hbm_gbps_algorithmic": round((16.0 * step_passes + 8.0 * readout_passes) * (1 << L) / (wall / args.steps) / 1e9, 1),
        "readout_ms": readout_ms, "readout_passes": readout_passes,
        "energy_density_last": e_series[-1],
        "roofline": roof,
    }
    # ---- the same step through the dense 6-qubit windows on the matrix cores
    variants = {}
    for var in DENSE:
        ev = fl.FloquetEngine(L, "c64", var)
        ev.set_xyz(w["J"], w["fields"], w["T"])
        ev.init(psi, w["spinors"])
        ev.step(psi, nblk)
        ev0.record(stream)
        for _ in range(reps):
            ev.step(psi, nblk)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / (nblk * reps)
        kind, fpa, mpeak = DENSE[var]
        nwin = sum(len(g) for g in _dense_groups(fl, L, nblk, kind)) * reps
        mflop = fpa * (1 << L) * nwin / (ev0.elapsed_time(ev1) / 1e3) / 1e12
        variants[var] = {"ms_per_period": round(ms, 3), "periods_per_s": round(1e3 / ms, 2),
                         "windows_per_period": nwin / (nblk * reps), "mfma_tflops": round(mflop, 2),
                         "mfma_peak": mpeak,
                         "energy_density_after_" + str(nblk * (reps + 1)): ev.energy_density(psi)}
        del ev
    out["dense_variants"] = variants
    del psi
    torch.cuda.empty_cache()
    if not args.no_adjoint:
        out["adjoint"] = adjoint_ratio(fl, torch)
        # the same ratio at L = 28 (2 GiB states; state, lambda and checkpoints far exceed the caches)
        out["adjoint_L28"] = adjoint_ratio(fl, torch, L=28)
        # the 4-qubit-window form: MFMA windows forward, their exact adjoints
        # replayed on the matrix cores
        out["adjoint_dense4"] = adjoint_ratio(fl, torch, variant="dense4_fp32")
        torch.cuda.empty_cache()
    if not args.no_l34:
        out["l34"] = l34_leg(fl, torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(L, args.cpu_sample_gates)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
