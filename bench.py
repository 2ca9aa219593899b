"""Benchmark of the compressed state-vector hot path on one MI355X.

Workload (default): n = 28 qubits, complex64 state held as compressed chunks of
2^20 amplitudes in HBM, error bound 1e-5 per component; circuit = QFT on a
seeded random basis state followed by 100 random one/two-qubit gates (520
gates). One step = init the basis state + apply the whole circuit (planning
of passes and fusion included: the plan is not reused between steps) as
streamed decode -> fused gates -> encode passes + the ZZ-chain expectation (an
FP64 reduction over the decoded state). Metric: amplitude-gate updates per
second including the codec = steps * gates * 2^n / time.

Prints one JSON line with the driver's fields plus "roofline" (the pass
kernel: algorithmic bytes per launch over its average launch duration, from
HIP events around every pass launch on the stream it runs on, against the HBM
bandwidth a copy kernel measures on the same device), "denominators" (the
measured HBM, host-link and matrix-core peaks) and "cpu_baseline" (the FP64
oracle on a bounded sample of the same circuit).

The compressed pass moves few bytes (about 10x fewer than the plain state),
so its HBM fraction is small: the pass is bound by vector-ALU issue (codec bit
planes, prefix sums, FP64 quantisation, gate arithmetic). That view is
reported beside the HBM one in roofline.alu: the library counts the
algorithmic lane operations of each pass in single-issue equivalents (FP32
gate arithmetic and 32-bit bit-plane ops count 1/2, since two of them issue
per slot); the peak is 256 CUs x 64 lanes x 2.4 GHz = 39.3 T of them per
second.

Other workloads (--workload): random20 (the small oracle-sized circuit),
host34 (n=34 state as compressed chunks in pinned host memory), adjoint22
(adjoint gradient of a 6-layer ansatz at n=22), batch256 (256 circuits of
12..24 qubits, plus 64 batched adjoint parameter sets at n=18). Each prints
its own JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_NOMINAL_GBS = 8000.0
VALU_PEAK_GOPS = 256 * 64 * 2.4   # single-issue lane operations per ns = Gop/s
MFMA_NOMINAL_TFLOPS = {"f32": 157.3, "bf16": 2500.0, "f64": 78.6}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=28)
    ap.add_argument("--eb", type=float, default=1e-5)
    ap.add_argument("--k", type=int, default=2)
    ap.add_argument("--mma", default="f32")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probes", action="store_true", help="skip the measured roofline denominators")
    ap.add_argument("--torch-runtime", action="store_true",
                    help="host34: run with PyTorch (and its copy of the HIP runtime) in the process")
    ap.add_argument("--cpu-share", type=float, default=0.0,
                    help="host34: also run with this share of chunk groups on host cores")
    ap.add_argument("--no-extras", action="store_true", help="skip comparison runs outside the timed loop")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--workload", default="qft28",
                    choices=["qft28", "random20", "host34", "host28", "adjoint22", "batch256", "table1"])
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device copy (scales the HBM byte counters)")
    return ap.parse_args()


# The complex64 compressed pass kernel that the counters in profiles/ cover:
# its launcher, its instantiation and every header it includes.
PASS_KERNEL_SOURCES = ("codec_device.h", "device_ops.h", "kernels.h", "mfma_ops.h", "pass_kernel.h", "reg_ops.h",
                       "tile_ops.h", "pass_kernel.hip", "pass_f32.hip")


def kernel_source_hash():
    """Hash of the sources of the headline pass kernel (the files above);
    other kernels and host-side planning code are not part of it."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2309_16979_amd", "csrc")
    for f in PASS_KERNEL_SOURCES:
        h.update(f.encode())
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(n_launch_bytes_key):
    """HBM bytes per pass launch from committed counter summaries, if they were
    taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "pass_kernel_qft28_counters.json")
    if not os.path.exists(p):
        return None
    try:
        doc = json.load(open(p))
    except Exception:
        return None
    if doc.get("kernel_hash") != kernel_source_hash():
        return None
    return doc.get(n_launch_bytes_key)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(n, x, gates, seconds):
    """FP64 oracle on the same circuit: gates applied in groups from |x> until
    about `seconds` of wall time (a bounded sample of the workload), on every
    host thread; then the same on one thread (a child process with
    OMP_NUM_THREADS=1, a third of the time)."""
    import subprocess
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    psi = oracle.basis(n, x)
    done = 0
    t0 = time.perf_counter()
    chunk = 4
    while done < len(gates):
        psi = oracle.simulate(n, gates[done:done + chunk], psi)
        done += len(gates[done:done + chunk])
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    del psi
    out = {"value": done * float(1 << n) / dt, "unit": "amplitude-gate updates/s",
           "cores": threads, "kind": "oracle", "cpu": cpu_model(),
           "sample": "FP64 uncompressed oracle simulator, first %d of %d gates of the same "
                     "n=%d circuit from the same basis state (%.1f s wall)" % (done, len(gates), n, dt)}
    code = ("import sys,time; sys.path.insert(0, %r); import oracle; from workloads import qft_plus_random; "
            "x, g = qft_plus_random(%d, 100, seed=%d); psi = oracle.basis(%d, x); t = time.perf_counter(); d = 0\n"
            "while d < len(g) and time.perf_counter() - t < %f:\n"
            "    psi = oracle.simulate(%d, g[d:d + 1], psi); d += 1\n"
            "print(d, time.perf_counter() - t)" % (ROOT, n, 0, n, seconds / 3.0, n))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
        d1, t1 = r.stdout.split()[-2:]
        out["one_thread"] = {"value": int(d1) * float(1 << n) / float(t1), "cores": 1,
                             "sample": "first %s gates (%.1f s wall)" % (d1, float(t1))}
    except Exception as e:   # reported, not fatal
        out["one_thread"] = {"error": str(e)}
    return out


def codec_cpu_baseline(n, eb, log2c=20, seconds=4.0):
    """The oracle's scalar codec (encode + decode of 2^log2c-amplitude complex64
    chunks with Gaussian components of an n-qubit random state) on one host
    thread and on every host thread (one chunk per call, calls on concurrent
    threads: ctypes releases the interpreter lock). GB/s of uncompressed
    amplitudes through encode and decode."""
    import concurrent.futures as cf
    import numpy as np
    import oracle
    rng = np.random.default_rng(5)
    sig = 2.0 ** (-(n + 1) / 2.0)
    chunk = (rng.standard_normal(1 << log2c) * sig + 1j * rng.standard_normal(1 << log2c) * sig).astype(np.complex64)

    def one():
        oracle.codec_decode(oracle.codec_encode(chunk, log2c, eb))

    res = {}
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    for th in (1, threads):
        done, t0 = 0, time.perf_counter()
        with cf.ThreadPoolExecutor(th) as ex:
            while time.perf_counter() - t0 < seconds / 2:
                list(ex.map(lambda _: one(), range(th)))
                done += th
        dt = time.perf_counter() - t0
        res["threads_%d" % th] = {"GBps": done * chunk.nbytes / dt / 1e9, "chunks": done, "s": dt}
    res["note"] = ("oracle scalar codec, complex64 chunks of 2^%d amplitudes, sigma 2^-%g, eb %g, encode + decode"
                   % (log2c, (n + 1) / 2.0, eb))
    return res


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(a state is not sharded across GPUs); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    if a.workload in ("host34", "host28") and not a.torch_runtime:
        # the library alone, on the HIP runtime it was built against: no
        # PyTorch in the process (host-store runs need no torch memory)
        os.environ["MSV_TORCH_RUNTIME"] = "0"
        (bench_host34 if a.workload == "host34" else bench_host28)(a)
        return
    import torch

    from paper_2309_16979_amd import Simulator, _lib
    from paper_2309_16979_amd.msv import probe_denominators
    from workloads import qft_plus_random, zz_chain

    if not os.path.exists(_lib.LIB_PATH):
        from paper_2309_16979_amd import build
        build.build()
    torch.cuda.set_device(0)
    if a.copy_probe:
        src = torch.ones(1 << 26, device="cuda")   # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel() * 4}))
        return
    if a.workload != "qft28":
        {"random20": bench_random20, "host34": bench_host34, "host28": bench_host28, "adjoint22": bench_adjoint22,
         "batch256": bench_batch256, "table1": bench_table1}[a.workload](a)
        return
    den = None if a.no_probes else probe_denominators()
    hbm_peak = den["hbm_copy_GBps"] if den else HBM_NOMINAL_GBS
    n = a.n
    x, gates = qft_plus_random(n, 100, seed=a.seed)
    masks, coeffs = zz_chain(n)
    G = len(gates)

    def run(sim):
        # the gates, then the Z-chain expectation, taken by the last pass
        sim.init_basis(x)
        return sim.apply_expect_z(gates, masks, coeffs)

    def timed_loop(sim, steps):
        acc = {"t_pass": 0.0, "passes": 0, "pass_bytes": 0, "pass_valu_ops": 0.0, "pass_issue_ops": 0.0,
               "pass_mfma_flops": 0.0}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            zz = run(sim)
            st = sim.stats()
            for k in acc:
                acc[k] += st[k]
        torch.cuda.synchronize()
        return time.perf_counter() - t0, zz, acc

    opts = {"time_passes": 1, "plan_cache": 0}
    if a.tile:
        opts["tile_qubits"] = a.tile
    sim = Simulator(n, dtype="c64", eb=a.eb, chunk_qubits=min(20, n), k_max=a.k, mma=a.mma, options=opts)
    for _ in range(a.warmup):
        run(sim)
    dt, zz, acc = timed_loop(sim, a.steps)
    value = a.steps * G * float(1 << n) / dt
    st = sim.stats()
    # the same loop with the plan of identical calls reused (the offline stage once)
    sim.set_option("plan_cache", 1)
    run(sim)
    dt_c, _, _ = timed_loop(sim, a.steps)

    n_pass = max(1, acc["passes"])
    avg_pass = acc["t_pass"] / n_pass
    bytes_per_pass = acc["pass_bytes"] / n_pass
    valu_per_pass = acc["pass_valu_ops"] / n_pass
    issue_per_pass = acc["pass_issue_ops"] / n_pass
    achieved_gbs = bytes_per_pass / avg_pass / 1e9 if avg_pass > 0 else 0.0
    achieved_gops = issue_per_pass / avg_pass / 1e9 if avg_pass > 0 else 0.0
    traffic = traffic_from_profiles("bytes_per_launch")
    roof = {"bound": "hbm", "achieved": round(achieved_gbs, 2), "peak": round(hbm_peak, 1), "unit": "GB/s",
            "frac": round(achieved_gbs / hbm_peak, 4), "traffic": traffic,
            "peak_source": "measured device copy kernel (msv_probe_hbm_copy)" if den else "nominal",
            "nominal_peak": HBM_NOMINAL_GBS,
            "kernel": "pass_kernel<float,%d,true,true,*,%d>" % (a.tile or 12, 0 if a.k < 3 else 1),
            "avg_launch_ms": round(avg_pass * 1e3, 4), "launches": acc["passes"],
            "algorithmic_bytes_per_launch": int(bytes_per_pass),
            "traffic_over_algorithmic": round(traffic / bytes_per_pass, 3) if traffic else None,
            "alu": {"achieved": round(achieved_gops, 1), "peak": round(VALU_PEAK_GOPS, 1),
                    "unit": "Gop/s (single-issue-equivalent vector lane operations)",
                    "frac": round(achieved_gops / VALU_PEAK_GOPS, 4),
                    "algorithmic_ops_per_launch": valu_per_pass,
                    "issue_equivalent_ops_per_launch": issue_per_pass}}
    if acc["pass_mfma_flops"] > 0 and avg_pass > 0:
        mk = {"f32": "mfma_f32_TFLOPs", "bf16": "mfma_bf16_TFLOPs", "f64": "mfma_f64_TFLOPs"}[a.mma]
        roof["mfma"] = {"achieved": round(acc["pass_mfma_flops"] / n_pass / avg_pass / 1e12, 3),
                        "peak": round(den[mk], 1) if den else MFMA_NOMINAL_TFLOPS[a.mma],
                        "nominal_peak": MFMA_NOMINAL_TFLOPS[a.mma], "unit": "TFLOP/s"}

    out = {"metric": "amplitude-gate updates/sec incl. codec", "value": value,
           "unit": "amplitude-gate updates/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": dt / a.steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "c64 (f32 gates, f64 codec quantisation and reductions)",
           "data": "synthetic: seeded QFT|x> + 100 random gates",
           "config": {"workload": "qft+100 random, n=%d, complex64, chunk 2^20, eb=%g, device store" % (n, a.eb),
                      "n": n, "gates": G, "eb": a.eb, "k_max": a.k, "mma": a.mma,
                      "passes": st["passes"], "fused_ops": st["fused_ops"], "planning": "every step",
                      "readout": "ZZ-chain expectation of the stored state, taken by the last pass"},
           "roofline": roof,
           "plan_reused": {"value": a.steps * G * float(1 << n) / dt_c, "ms_per_step": dt_c / a.steps * 1e3,
                           "note": "same loop with option plan_cache=1 (passes and fusion planned once)"}}
    if den:
        out["denominators"] = den
    out["compression"] = {"ratio": st["ratio"], "qubits_gained": math.log2(st["ratio"]) if st["ratio"] > 0 else None,
                          "compressed_bytes": st["compressed_bytes"], "reserved_bytes": st["reserved_bytes"],
                          "uncompressed_bytes": st["uncompressed_bytes"],
                          "reserved_over_uncompressed": st["reserved_bytes"] / st["uncompressed_bytes"],
                          "max_err_all": st["max_err_all"],
                          "err_bound": st["err_bound"], "bound_violations": st["bound_violations"],
                          "zz_expectation": zz}
    sim.close()

    if not a.no_extras:
        # fidelity against an FP64 (complex128, uncompressed) run on the same GPU
        ref = Simulator(n, dtype="c128", eb=0.0, k_max=a.k)
        t1 = time.perf_counter()
        run(ref)
        torch.cuda.synchronize()
        t_ref = time.perf_counter() - t1
        amps_ref = ref.amplitudes()
        ref.close()
        sim = Simulator(n, dtype="c64", eb=a.eb, chunk_qubits=min(20, n), k_max=a.k, mma=a.mma)
        run(sim)
        fr, fn = sim.fidelity(amps_ref)
        sim.close()
        plain = Simulator(n, dtype="c64", eb=0.0, k_max=a.k, mma=a.mma, options={"time_passes": 1})
        run(plain)
        t1 = time.perf_counter()
        run(plain)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t1
        pst = plain.stats()
        plain.close()
        out["fidelity_vs_fp64"] = {"f_raw": fr, "f_norm": fn, "reference": "complex128 uncompressed GPU run"}
        # fused width k on the matrix cores (FP32 / BF16 inputs), same workload
        sweep = {}
        for k, mma in ((3, "f32"), (4, "f32"), (5, "f32"), (4, "bf16"), (5, "bf16")):
            sm = Simulator(n, dtype="c64", eb=a.eb, chunk_qubits=min(20, n), k_max=k, mma=mma)
            run(sm)
            t1 = time.perf_counter()
            run(sm)
            torch.cuda.synchronize()
            dtk = time.perf_counter() - t1
            fk = sm.fidelity(amps_ref)
            stk = sm.stats()
            sm.close()
            sweep["k%d_%s" % (k, mma)] = {"updates_per_s": G * float(1 << n) / dtk, "f_norm": fk[1],
                                          "mfma_ops": stk["mfma_ops"], "fused_ops": stk["fused_ops"]}
        out["mfma_sweep"] = sweep
        # codec predictor mode 1 (per-block choice), same workload: the same
        # decoded state, fewer bytes, more encode work
        sp = Simulator(n, dtype="c64", eb=a.eb, chunk_qubits=min(20, n), k_max=a.k, mma=a.mma,
                       options={"predictor": 1})
        run(sp)
        t1 = time.perf_counter()
        run(sp)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - t1
        stp = sp.stats()
        fp = sp.fidelity(amps_ref)
        sp.close()
        out["predictor_mode1"] = {"updates_per_s": G * float(1 << n) / dtp, "ratio": stp["ratio"],
                                  "compressed_bytes": stp["compressed_bytes"], "f_norm": fp[1],
                                  "ratio_mode0": st["ratio"]}
        del amps_ref
        plain_gbs = pst["pass_bytes"] / pst["t_pass"] / 1e9 if pst["t_pass"] else None
        out["comparators"] = {
            "c64_uncompressed_updates_per_s": G * float(1 << n) / t_plain,
            "c64_uncompressed_pass_GBps": plain_gbs,
            "c64_uncompressed_pass_hbm_frac": plain_gbs / hbm_peak if plain_gbs else None,
            "c128_uncompressed_updates_per_s": G * float(1 << n) / t_ref,
        }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, x, gates, a.cpu_seconds)
        out["cpu_baseline"]["codec"] = codec_cpu_baseline(n, a.eb)
    print(json.dumps(out), flush=True)


def _timed(fn, reps):
    """Wall time per call of fn (every library call returns with its work
    finished; with torch in the process its queues are drained as well)."""
    sync = None
    if os.environ.get("MSV_TORCH_RUNTIME", "1") != "0":
        import torch
        sync = torch.cuda.synchronize
    if sync:
        sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        r = fn()
    if sync:
        sync()
    return (time.perf_counter() - t0) / reps, r


def bench_random20(a):
    """n=20 complex128, random depth-20 circuit from |0>, 2^14-amplitude
    chunks: uncompressed and eb=1e-4; the FP64 oracle on all host threads and
    on one thread (the whole circuit), and the fidelity of each GPU run."""
    import numpy as np
    import oracle
    from paper_2309_16979_amd import Simulator
    from workloads import random_circuit
    n = 20
    gates = random_circuit(n, 20, seed=a.seed)
    out = {"metric": "amplitude-gate updates/sec incl. codec", "unit": "amplitude-gate updates/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "c128", "data": "synthetic: seeded random circuit",
           "config": {"workload": "random depth 20, n=20, complex128, chunk 2^14", "gates": len(gates)}}
    t0 = time.perf_counter()
    ref = oracle.simulate(n, gates, 0)
    t_or = time.perf_counter() - t0
    for eb in (0.0, 1e-4):
        with Simulator(n, dtype="c128", eb=eb, chunk_qubits=14) as s:
            def run():
                s.init_basis(0)
                s.apply(gates)
            run()
            dt, _ = _timed(run, max(5, a.steps))
            st = s.stats()
            f = s.fidelity(ref)
            out["eb=%g" % eb] = {"updates_per_s": len(gates) * float(1 << n) / dt, "s_per_apply": dt,
                                 "passes": st["passes"], "ratio": st["ratio"], "f_raw": f[0], "f_norm": f[1],
                                 "max_err_all": st["max_err_all"], "bound_violations": st["bound_violations"]}
    out["value"] = out["eb=0.0001"]["updates_per_s"]
    out["oracle"] = {"threads": int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count(),
                     "updates_per_s": len(gates) * float(1 << n) / t_or}
    env = dict(os.environ, OMP_NUM_THREADS="1")
    import subprocess
    code = ("import sys,time; sys.path.insert(0, %r); import oracle; from workloads import random_circuit; "
            "g = random_circuit(20, 20, seed=%d); t = time.perf_counter(); oracle.simulate(20, g, 0); "
            "print(len(g) * 2.0 ** 20 / (time.perf_counter() - t))" % (ROOT, a.seed))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    out["oracle_1_thread_updates_per_s"] = float(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 else None
    print(json.dumps(out), flush=True)


def bench_host28(a):
    """The headline circuit (QFT|x> + 100 random gates, n=28, complex64,
    eb=1e-5, chunks of 2^20 amplitudes) on the host-pinned store: the same
    compressed passes, with the chunks streamed from pinned host memory over
    the host link (the configuration's second store)."""
    from paper_2309_16979_amd import Simulator
    from workloads import qft_plus_random
    use_torch = os.environ.get("MSV_TORCH_RUNTIME", "1") != "0"
    n, log2c, eb = 28, 20, 1e-5
    x, gates = qft_plus_random(n, 100, seed=a.seed)
    with Simulator(n, dtype="c64", eb=eb, chunk_qubits=log2c, store="host", k_max=a.k, use_torch=use_torch) as s:
        def run():
            s.init_basis(x)
            s.apply(gates)
        run()
        dt, _ = _timed(run, max(1, a.steps))
        st = s.stats()
    link_bytes = st["h2d_bytes"] + st["d2h_bytes"]
    out = {"metric": "amplitude-gate updates/sec incl. codec and host link", "unit": "amplitude-gate updates/s",
           "value": len(gates) * float(1 << n) / dt, "n_gpus": 1, "higher_is_better": True, "dtype": "c64",
           "data": "synthetic: seeded QFT|x> + 100 random gates",
           "config": {"workload": "qft+100 random, n=28, complex64, chunk 2^20, eb=1e-05, host-pinned store",
                      "gates": len(gates), "pytorch_in_process": use_torch},
           "s_per_apply": dt, "passes": st["passes"], "ratio": st["ratio"],
           "bound_violations": st["bound_violations"],
           "host_link": {"h2d_bytes": st["h2d_bytes"], "d2h_bytes": st["d2h_bytes"], "overlap": st["overlap"],
                         "t_kernel": st["t_kernel"], "link_GBps_over_apply": link_bytes / dt / 1e9,
                         "zero_groups_skipped": st["zero_groups_skipped"]}}
    print(json.dumps(out), flush=True)


def bench_host34(a):
    """n=34 complex64 held as compressed 2^22-amplitude chunks in pinned host
    memory (128 GiB uncompressed); random depth-40 circuit with 30% two-qubit
    gates on qubits that cross chunks; plus GHZ-34 (exact). Two error bounds:
    the configuration's absolute eb = 1e-4, which is larger than the
    amplitudes of the spread state (about 5.4e-6 per component) and collapses
    it to ZERO chunks, and a norm-relative eb = 0.1 x 2^-17 = 7.6e-7, which
    keeps the state (the headline of this workload)."""
    from paper_2309_16979_amd import Simulator
    from workloads import crossing_circuit, ghz
    use_torch = os.environ.get("MSV_TORCH_RUNTIME", "1") != "0"
    n, log2c = 34, 22
    gates = crossing_circuit(n, 40, log2c, seed=a.seed)
    out = {"metric": "amplitude-gate updates/sec incl. codec and host link", "unit": "amplitude-gate updates/s",
           "n_gpus": 1, "higher_is_better": True, "data": "synthetic: seeded random circuit, crossing 2q gates",
           "dtype": "c64", "config": {"workload": "random depth 40, 30% crossing 2q gates, n=34, complex64, "
                                      "chunk 2^22, host-pinned store; eb norm-relative 0.1 (and absolute 1e-4)",
                                      "gates": len(gates), "pytorch_in_process": use_torch}}
    den = None
    if not a.no_probes:
        from paper_2309_16979_amd.msv import probe_denominators
        den = probe_denominators()
        out["denominators"] = den
    runs = [("eb_rel_0.1", 0.1, "rel", {}), ("eb_abs_1e-4", 1e-4, "abs", {})]
    if a.cpu_share > 0:
        runs.append(("eb_rel_0.1_cpu_share", 0.1, "rel", {"cpu_share": a.cpu_share, "cpu_threads": 8}))
    for tag, eb, mode, opts in runs:
        with Simulator(n, dtype="c64", eb=eb, eb_mode=mode, chunk_qubits=log2c, store="host", k_max=a.k,
                       options=opts, use_torch=use_torch) as s:
            def run():
                s.init_basis(0)
                s.apply(gates)
            reps = max(1, a.steps) if tag == "eb_rel_0.1" else 1
            dt, _ = _timed(run, reps)
            st = s.stats()
            link_bytes = st["h2d_bytes"] + st["d2h_bytes"]
            r = {"updates_per_s": len(gates) * float(1 << n) / dt, "s_per_apply": dt, "steps": reps,
                 "eb": st["err_bound"],
                 "host_link": {"h2d_GBps": st["h2d_bytes"] / st["t_h2d"] / 1e9 if st["t_h2d"] else None,
                               "d2h_GBps": st["d2h_bytes"] / st["t_d2h"] / 1e9 if st["t_d2h"] else None,
                               "h2d_bytes": st["h2d_bytes"], "d2h_bytes": st["d2h_bytes"],
                               "overlap": st["overlap"], "t_kernel": st["t_kernel"], "t_total": st["t_total"],
                               "passes": st["passes"], "zero_groups_skipped": st["zero_groups_skipped"],
                               "cpu_groups": st["cpu_groups"],
                               "link_GBps_over_apply": link_bytes / dt / 1e9},
                 "compression": {"ratio": st["ratio"], "compressed_bytes": st["compressed_bytes"],
                                 "reserved_bytes": st["reserved_bytes"], "max_err_all": st["max_err_all"],
                                 "err_bound": st["err_bound"], "bound_violations": st["bound_violations"]}}
            if den:
                # the link roofline: both directions at once (bidirectional probe)
                r["host_link"]["frac_of_bidir_peak"] = link_bytes / dt / 1e9 / den["bidir_GBps"]
            out[tag] = r
            print("host34 %s: %.2f s per apply, ratio %.1f" % (tag, dt, st["ratio"]), file=sys.stderr, flush=True)
    out["value"] = out["eb_rel_0.1"]["updates_per_s"]
    with Simulator(n, dtype="c64", eb=1e-4, chunk_qubits=log2c, store="host", use_torch=use_torch) as s:
        s.init_basis(0)
        t0 = time.perf_counter()
        s.apply(ghz(n))
        t_ghz = time.perf_counter() - t0
        amp0 = s.amplitudes(0, 1)[0]
        amp1 = s.amplitudes((1 << n) - 1, 1)[0]
        out["ghz34"] = {"amp_0": [float(amp0.real), float(amp0.imag)], "amp_last": [float(amp1.real), float(amp1.imag)],
                        "expected": 2 ** -0.5, "p_one_q0": s.prob_one(0), "s": t_ghz}
    print(json.dumps(out), flush=True)


def bench_adjoint22(a):
    """Adjoint gradient, n=22 complex64, hardware-efficient ansatz (6 layers of
    RY RZ on every qubit + CZ ring), observable sum Z_i Z_(i+1), compressed
    checkpoints every 2 layers (uncompressed and eb=1e-4 states)."""
    import numpy as np
    from paper_2309_16979_amd import Simulator
    from workloads import ansatz, ansatz_params, zz_chain
    n, layers = 22, 6
    gates = ansatz(n, layers)
    params = ansatz_params(n, layers, seed=a.seed)[0]
    masks, coeffs = zz_chain(n)
    per_layer = len(gates) // layers
    ck = [2 * per_layer, 4 * per_layer]
    out = {"metric": "adjoint gradients/s", "unit": "gradients/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": "c64", "data": "synthetic: seeded ansatz parameters",
           "config": {"workload": "ansatz n=22, 6 layers RY RZ + CZ ring, ZZ chain, checkpoints every 2 layers",
                      "gates": len(gates), "params": int(params.size)}}
    for eb in (0.0, 1e-4):
        with Simulator(n, dtype="c64", eb=eb, chunk_qubits=16) as s:
            def run():
                s.init_basis(0)
                return s.adjoint(gates, params, masks, coeffs, ck)
            run()
            dt, (ev, grad) = _timed(run, max(1, a.steps))
            # gate applications: forward + recompute of each segment + two sweeps of U^dagger
            apps = 4 * len(gates)
            out["eb=%g" % eb] = {"s_per_gradient": dt, "gradients_per_s": 1.0 / dt, "energy": ev,
                                 "updates_per_s": apps * float(1 << n) / dt,
                                 "grad_norm": float(np.linalg.norm(grad))}
    out["value"] = out["eb=0"]["gradients_per_s"]
    print(json.dumps(out), flush=True)


def bench_batch256(a):
    """256 circuits of n ~ U{12..24}, depth ~ U{10..60}, complex64, eb=1e-4,
    autotuned fusion width and tile; plus 64 ansatz parameter sets at n=18
    through the batched adjoint."""
    import numpy as np
    from paper_2309_16979_amd import msv
    from workloads import ansatz, ansatz_params, batch_circuits, zz_chain
    circuits = [(n, g, 0) for n, g in batch_circuits(256, seed=a.seed)]
    upd = sum(len(g) * float(1 << n) for n, g, _ in circuits)
    msv.batch_run(circuits, dtype="c64", eb=1e-4)
    dt, (st, _) = _timed(lambda: msv.batch_run(circuits, dtype="c64", eb=1e-4), max(1, a.steps))
    out = {"metric": "amplitude-gate updates/sec incl. codec (batched)", "unit": "amplitude-gate updates/s",
           "value": upd / dt, "n_gpus": 1, "higher_is_better": True, "dtype": "c64",
           "data": "synthetic: seeded random circuits",
           "config": {"workload": "256 circuits n in [12,24], depth 10..60, complex64, eb=1e-4, autotuned",
                      "circuits": 256, "updates": upd},
           "s_per_batch": dt, "kernel_launches": st["kernel_launches"], "passes": st["passes"],
           "kernel_s": st["t_kernel"], "note": "s_per_batch is the whole call: simulators, planning (cost-model "
           "search on the host), upload, the persistent launch and read-back; kernel_s is the launch alone"}
    n, layers, sets = 18, 6, 64
    gates = ansatz(n, layers)
    P = ansatz_params(n, layers, seed=a.seed, count=sets)
    masks, coeffs = zz_chain(n)
    msv.batch_adjoint(n, gates, P[:2], masks, coeffs)
    dt2, _ = _timed(lambda: msv.batch_adjoint(n, gates, P, masks, coeffs), 1)
    out["batched_adjoint"] = {"sets": sets, "n": n, "s": dt2, "gradients_per_s": sets / dt2}
    print(json.dumps(out), flush=True)


# The paper's Table 1 (its only measurements): whole-state host<->GPU transfer
# time in seconds, (H2D, D2H), on its own unnamed CUDA GPU and host, precision
# and memory kind not stated. Quoted as context.
PAPER_TABLE1 = {20: {"sync": (0.003, 0.008), "per_amplitude": (2.7, 9.2), "staged_remap": (0.003, 0.004)},
                25: {"sync": (0.080, 0.233), "per_amplitude": (77.9, 294.4), "staged_remap": (0.110, 0.273)}}


def bench_table1(a):
    """The paper's transfer experiment on this MI355X: a complex128 state of
    2^20 and 2^25 amplitudes moved host->GPU and GPU->host by one whole-state
    copy, by one asynchronous copy per amplitude (a bounded sample of 2^15
    calls, extrapolated) and by a bulk copy into a staging buffer plus a GPU
    kernel that places every amplitude; pinned and pageable host memory."""
    from paper_2309_16979_amd.msv import probe_transfer
    rows = {}
    for n in (20, 25):
        for strat in ("sync", "per_amplitude", "staged_remap"):
            for pinned in (True, False):
                for to_dev in (True, False):
                    r = probe_transfer(n, strat, to_dev, pinned)
                    print("table1 n=%d %s %s %s: %.4f s" % (n, strat, "pinned" if pinned else "pageable",
                                                             "h2d" if to_dev else "d2h", r["seconds"]),
                          file=sys.stderr, flush=True)
                    key = "n%d_%s_%s_%s" % (n, strat, "pinned" if pinned else "pageable", "h2d" if to_dev else "d2h")
                    r["GBps"] = 16.0 * (1 << n) / r["seconds"] / 1e9
                    r["paper_seconds"] = PAPER_TABLE1[n][strat][0 if to_dev else 1]
                    rows[key] = r
    s20 = rows["n20_sync_pinned_h2d"]["seconds"]
    out = {"metric": "whole-state host<->GPU transfer time (paper Table 1)", "unit": "s", "n_gpus": 1,
           "higher_is_better": False, "dtype": "c128", "data": "synthetic: index-pattern state",
           "value": rows["n25_staged_remap_pinned_h2d"]["seconds"],
           "config": {"workload": "paper Table 1: n=20 and 25, complex128, sync / per-amplitude async / "
                                  "staged buffer + GPU remap, pinned and pageable"},
           "rows": rows,
           "ratios_n20_pinned": {"per_amplitude_over_sync": rows["n20_per_amplitude_pinned_h2d"]["seconds"] / s20,
                                 "staged_over_sync": rows["n20_staged_remap_pinned_h2d"]["seconds"] / s20},
           "paper_context": "Table 1 of the paper, its own GPU (unnamed CUDA device), quoted per row as "
                            "paper_seconds"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
