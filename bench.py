"""Benchmark of the compressed state-vector hot path on one MI355X.

Workload (default): n = 28 qubits, complex64 state held as compressed chunks of
2^20 amplitudes in HBM, error bound 1e-5 per component; circuit = QFT on a
seeded random basis state followed by 100 random one/two-qubit gates (520
gates). One step = init the basis state + apply the whole circuit as streamed
decode -> fused gates -> encode passes + the ZZ-chain expectation (an FP64
reduction over the decoded state). Metric: amplitude-gate updates per second
including the codec = steps * gates * 2^n / time.

Prints one JSON line with the driver's fields plus "roofline" (pass kernel,
durations from HIP events around every pass launch on the stream it runs on)
and "cpu_baseline" (the FP64 oracle on a bounded sample of the same circuit).
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

HBM_PEAK_GBS = 8000.0


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
    ap.add_argument("--no-extras", action="store_true", help="skip comparison runs outside the timed loop")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    return ap.parse_args()


def kernel_source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2309_16979_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
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


def cpu_baseline(n, x, gates, seconds):
    """FP64 oracle on the same circuit: gates applied one by one from |x> until
    about `seconds` of CPU time (a bounded sample of the workload)."""
    import numpy as np
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
    return {"value": done * float(1 << n) / dt, "unit": "amplitude-gate updates/s",
            "cores": threads, "kind": "oracle",
            "sample": "FP64 uncompressed oracle simulator, first %d of %d gates of the same "
                      "n=%d circuit from the same basis state (%.1f s wall)" % (done, len(gates), n, dt)}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(sharding is described in DESIGN.md); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2309_16979_amd import Simulator, _lib
    from workloads import qft_plus_random, zz_chain

    if not os.path.exists(_lib.LIB_PATH):
        from paper_2309_16979_amd import build
        build.build()
    torch.cuda.set_device(0)
    n = a.n
    x, gates = qft_plus_random(n, 100, seed=a.seed)
    masks, coeffs = zz_chain(n)
    G = len(gates)

    def run(sim):
        sim.init_basis(x)
        sim.apply(gates)
        return sim.expect_z(masks, coeffs)

    opts = {"time_passes": 1}
    if a.tile:
        opts["tile_qubits"] = a.tile
    sim = Simulator(n, dtype="c64", eb=a.eb, chunk_qubits=min(20, n), k_max=a.k, mma=a.mma, options=opts)
    for _ in range(a.warmup):
        run(sim)
    torch.cuda.synchronize()
    t_pass = 0.0
    n_pass = 0
    pass_bytes = 0
    t0 = time.perf_counter()
    for _ in range(a.steps):
        zz = run(sim)
        st = sim.stats()
        t_pass += st["t_pass"]
        n_pass += st["passes"]
        pass_bytes += st["pass_bytes"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = a.steps * G * float(1 << n) / dt
    st = sim.stats()

    avg_pass = t_pass / max(1, n_pass)
    bytes_per_pass = pass_bytes / max(1, n_pass)
    achieved = bytes_per_pass / avg_pass / 1e9 if avg_pass > 0 else 0.0
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_from_profiles("bytes_per_launch"),
            "kernel": "pass_kernel<float,%d,true,true>" % (a.tile or 12),
            "avg_launch_ms": round(avg_pass * 1e3, 4), "launches": n_pass,
            "algorithmic_bytes_per_launch": int(bytes_per_pass)}

    out = {"metric": "amplitude-gate updates/sec incl. codec", "value": value,
           "unit": "amplitude-gate updates/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": dt / a.steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "c64 (f32 gates, f64 codec quantisation and reductions)",
           "data": "synthetic: seeded QFT|x> + 100 random gates",
           "config": {"workload": "qft+100 random, n=%d, complex64, chunk 2^20, eb=%g, device store" % (n, a.eb),
                      "n": n, "gates": G, "eb": a.eb, "k_max": a.k, "mma": a.mma,
                      "passes": st["passes"], "fused_ops": st["fused_ops"]},
           "roofline": roof}
    out["compression"] = {"ratio": st["ratio"], "qubits_gained": math.log2(st["ratio"]) if st["ratio"] > 0 else None,
                          "compressed_bytes": st["compressed_bytes"], "max_err_all": st["max_err_all"],
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
        del amps_ref
        plain = Simulator(n, dtype="c64", eb=0.0, k_max=a.k, mma=a.mma, options={"time_passes": 1})
        run(plain)
        t1 = time.perf_counter()
        run(plain)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t1
        pst = plain.stats()
        plain.close()
        out["fidelity_vs_fp64"] = {"f_raw": fr, "f_norm": fn, "reference": "complex128 uncompressed GPU run"}
        out["comparators"] = {
            "c64_uncompressed_updates_per_s": G * float(1 << n) / t_plain,
            "c64_uncompressed_pass_GBps": pst["pass_bytes"] / pst["t_pass"] / 1e9 if pst["t_pass"] else None,
            "c128_uncompressed_updates_per_s": G * float(1 << n) / t_ref,
        }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, x, gates, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
