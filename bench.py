"""Benchmark: dd Rgemm on one MI355X, plain and split forms, plus served latency.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 8192] [--no-cpu]
                    [--sections plain,sizes,syrk,cgemm,potrf,qd,ozaki,host,serve]

One step = one dd Rgemm NN, m = n = k = n (8192), leading dimensions 8195,
C <- alpha*A*B + beta*C on float64 hi/lo planes already resident in HBM.
The headline value is dd-GFLOPS = 2*m*n*k / time (one dd multiply-add = two
dd flops), over exactly K timed steps bracketed by device synchronisations.
Prints ONE JSON line.  Extra sections report the other Rgemm sizes, Rsyrk,
Cgemm, the Cholesky Rpotrf, the quad-double Rgemm, the split forms, the
host-pointer call and the served request stream, with the same input recipes;
the CPU oracle is timed on a bounded sample of the headline product.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "dd-GFLOPS Rgemm n=8192 (plain vs Ozaki-split); served p50/p99 latency"
FP64_PEAK_TFLOPS = 78.6          # MI355X FP64 vector peak (FMA = 2 flops)
HBM_PEAK_GBS = 8000.0
INT8_PEAK_TOPS = 5000.0          # dense INT8 matrix peak, ops/s (MAC = 2 ops)
OPS_PER_MADD_ALG = 20            # FP64 issue slots per dd multiply-add (roofline unit)
OPS_PER_MADD_LEAN = 10           # what the plain kernel issues per dd multiply-add (8 vector + 2 MFMA)
KERNEL_SOURCES = ["paper_2109_13406_amd/csrc/gemm_plain.hip", "paper_2109_13406_amd/csrc/dd.hpp",
                  "paper_2109_13406_amd/build.py"]    # (its per-source flags shape the kernel)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sha():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def timed_calls(fn, steps, warmup, stream):
    """Warm up, then time exactly `steps` calls with HIP events on `stream`
    (the stream the library launches on).  Returns (total_s, per_call_s list)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    evs[0].record(stream)
    for i in range(steps):
        fn()
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    per = [evs[i].elapsed_time(evs[i + 1]) / 1e3 for i in range(steps)]
    return total, per


def traffic_record(name):
    """HBM traffic of the dominant kernel from the committed rocprofv3 counter
    summary, or None if it is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_sha") != kernel_sha():
        return None
    return rec.get("bytes_per_launch")


def bench_plain(h, args, stream):
    import torch
    import workloads as W
    from paper_2109_13406_amd import binding as b
    n = args.n
    case = W.gemm_case_device(W.BASE_SEED + 1, "N", "N", n, n, n)
    A, B, C = case["A"], case["B"], case["C"]
    torch.cuda.synchronize()

    opts = dict(algo=b.MPDD_PLAIN, tile_id=args.tile, splitk=0)

    def step():
        info = b.mpdd_Rgemm_ex(h, opts, "N", "N", n, n, n, case["alpha"], A, case["lda"], B,
                               case["ldb"], case["beta"], C, case["ldc"], stream=stream)
        if info != 0:
            raise RuntimeError(f"mpdd_Rgemm info={info}")

    total, per = timed_calls(step, args.steps, args.warmup, stream)
    return case, total, per


def bench_sizes(h, args, stream):
    """The other products of the Rgemm size sweep (square NN and TN at
    1024 .. 4096, the 4096 x 4096 x 256 and 8192 x 64 x 8192 shapes), default
    tile and k-split choice, padded leading dimensions."""
    import torch
    import workloads as W
    from paper_2109_13406_amd import binding as b
    out = []
    for (ta, tb, m, n, k) in (("N", "N", 1024, 1024, 1024), ("N", "N", 2048, 2048, 2048),
                              ("N", "N", 4096, 4096, 4096), ("T", "N", 4096, 4096, 4096),
                              ("N", "T", 4096, 4096, 4096), ("T", "T", 4096, 4096, 4096),
                              ("N", "N", 4096, 4096, 256), ("N", "N", 8192, 64, 8192)):
        case = W.gemm_case_device(W.BASE_SEED + 1, ta, tb, m, n, k)
        torch.cuda.synchronize()

        def step():
            info = b.mpdd_Rgemm(h, ta, tb, m, n, k, case["alpha"], case["A"], case["lda"],
                                case["B"], case["ldb"], case["beta"], case["C"], case["ldc"],
                                stream=stream)
            if info != 0:
                raise RuntimeError(f"mpdd_Rgemm info={info}")
        _, per = timed_calls(step, 3, 1, stream)
        t = sum(per) / len(per)
        out.append({"op": ta + tb, "m": m, "n": n, "k": k, "ms": round(t * 1e3, 3),
                    "dd_gflops": round(2.0 * m * n * k / t / 1e9, 1)})
        log(f"size {out[-1]}")
        del case
        torch.cuda.empty_cache()
    return out


def cpu_baseline(case, n, cols=64):
    """Time the CPU oracle (as it stands) on all m rows x `cols` columns of the
    same product: A and the selected B columns copied to the host."""
    import numpy as np
    import oracle
    ncores = len(os.sched_getaffinity(0))
    A = tuple(x.cpu().numpy() for x in case["A"])
    ldb = case["ldb"]
    Bc = tuple(np.ascontiguousarray(x[: ldb * cols].cpu().numpy()) for x in case["B"])
    C = tuple(np.zeros(n * cols) for _ in range(2))
    t0 = time.perf_counter()
    info = oracle.rgemm("N", "N", n, cols, n, case["alpha"], A, case["lda"], Bc, ldb, (0.0, 0.0),
                        C, n)
    dt = time.perf_counter() - t0
    assert info == 0
    return {"value": round(2.0 * n * cols * n / dt / 1e9, 3), "unit": "dd-GFLOPS",
            "cores": ncores, "kind": "oracle",
            "sample": f"Rgemm NN m={n} n={cols} k={n} (the first {cols} columns of the "
                      f"timed product), beta=0, {dt:.2f} s wall, OpenMP threads={ncores}"}


def bench_syrk(h, args, stream):
    import torch
    import workloads as W
    from paper_2109_13406_amd import binding as b
    n = args.n
    case = W.syrk_case_device(W.BASE_SEED + 2, "U", "N", n, n)
    torch.cuda.synchronize()

    def step():
        info = b.mpdd_Rsyrk(h, "U", "N", n, n, case["alpha"], case["A"], case["lda"],
                            case["beta"], case["C"], case["ldc"], stream=stream)
        if info != 0:
            raise RuntimeError(f"mpdd_Rsyrk info={info}")

    total, per = timed_calls(step, max(1, args.steps // 2), 1, stream)
    t = sum(per) / len(per)
    flops = float(n) * (n + 1) * n
    del case
    torch.cuda.empty_cache()
    return {"workload": f"Rsyrk U N n={n} k={n} ld={W.ld_padded(n)}", "ms": round(t * 1e3, 3),
            "dd_gflops": round(flops / t / 1e9, 1)}


def bench_cgemm(h, args, stream):
    """Complex dd Cgemm NN at n/2, four-product (default) and three-product
    forms.  Complex flops: 8 mnk (LAWN 41: 6 real multiplies + 2 adds per
    complex multiply-add), for both forms."""
    import torch
    import workloads as W
    from paper_2109_13406_amd import binding as b
    n = max(1, args.n // 2)
    case = W.cgemm_case_device(W.BASE_SEED + 5, "N", "N", n, n, n)
    torch.cuda.synchronize()
    out = {"workload": f"Cgemm NN m=n=k={n} ld={W.ld_padded(n)} (four real dd planes each)"}
    for form, opts in (("4m", None), ("3m", dict(algo=b.MPDD_COMPLEX_3M))):
        def step():
            info = b.mpdd_Cgemm_ex(h, opts, "N", "N", n, n, n, case["alpha"], case["A"],
                                   case["lda"], case["B"], case["ldb"], case["beta"], case["C"],
                                   case["ldc"], stream=stream)
            if info != 0:
                raise RuntimeError(f"mpdd_Cgemm_ex info={info}")

        total, per = timed_calls(step, max(1, args.steps // 2), 1, stream)
        t = sum(per) / len(per)
        out[f"ms_{form}"] = round(t * 1e3, 3)
        out[f"complex_dd_gflops_{form}"] = round(8.0 * n ** 3 / t / 1e9, 1)
    del case
    torch.cuda.empty_cache()
    return out


def bench_potrf(h, args, stream):
    """Blocked dd Cholesky Rpotrf L at n (synchronous call: it reads each
    diagonal block's info back).  dd-flops n^3/3 (LAWN 41, leading term)."""
    import torch
    import workloads as W
    from paper_2109_13406_amd import binding as b
    n = args.n
    case = W.spd_case_device(W.BASE_SEED + 7, n, "L")
    A0 = tuple(x.clone() for x in case["A"])
    torch.cuda.synchronize()
    times = []
    for rep in range(1 + max(1, args.steps // 2)):
        for dst, src in zip(case["A"], A0):
            dst.copy_(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, info = b.mpdd_Rpotrf(h, "L", n, case["A"], case["lda"], stream=stream)
        torch.cuda.synchronize()
        if rc != 0 or info != 0:
            raise RuntimeError(f"mpdd_Rpotrf rc={rc} info={info}")
        if rep > 0:                      # the first call is warm-up
            times.append(time.perf_counter() - t0)
    t = sum(times) / len(times)
    del case, A0
    torch.cuda.empty_cache()
    return {"workload": f"Rpotrf L n={n} ld={W.ld_padded(n)} (SPD: dd U[-1,1) off-diagonal, "
                        f"n + U[0,1) diagonal)", "ms": round(t * 1e3, 3),
            "dd_gflops": round(float(n) ** 3 / 3.0 / t / 1e9, 1)}


def bench_qd(h, args, stream):
    """Quad-double Rgemm NN at n/4 (four planes per matrix; ~10x the binary64
    work of a dd multiply-add).  qd-flops 2mnk."""
    import torch
    import workloads as W
    from paper_2109_13406_amd import binding as b
    n = max(1, args.n // 4)
    g = torch.Generator(device="cuda")
    g.manual_seed(W.BASE_SEED + 9)
    ld = W.ld_padded(n)

    def qmat():
        x0 = torch.rand(ld * n, generator=g, dtype=torch.float64, device="cuda") * 2 - 1
        parts = [x0]
        for _ in range(3):
            u = torch.rand(ld * n, generator=g, dtype=torch.float64, device="cuda") * 2 - 1
            parts.append(parts[-1] * 2.0 ** -54 * u)
        return tuple(parts)
    A, B, C = qmat(), qmat(), qmat()
    alpha, beta = (0.75, 2.0 ** -60, 0.0, 0.0), (-0.5, 0.0, 0.0, 0.0)
    torch.cuda.synchronize()

    def step():
        info = b.mpdd_Qgemm(h, "N", "N", n, n, n, alpha, A, ld, B, ld, beta, C, ld, stream=stream)
        if info != 0:
            raise RuntimeError(f"mpdd_Qgemm info={info}")

    total, per = timed_calls(step, max(1, args.steps // 2), 1, stream)
    t = sum(per) / len(per)
    del A, B, C
    torch.cuda.empty_cache()
    return {"workload": f"Qgemm NN m=n=k={n} ld={ld} (quad-double, four binary64 planes each)",
            "ms": round(t * 1e3, 3), "qd_gflops": round(2.0 * n ** 3 / t / 1e9, 1)}


def ratio_gpu(C, R, m, n, ldc, k):
    """Normwise dd difference of the stored m x n entries of C from R in units
    of k * 2^-104, on the device (the tests' metric: (hi - hi') + (lo - lo'))."""
    import torch
    C = tuple(x[: ldc * n].view(n, ldc)[:, :m] for x in C)
    R = tuple(x[: ldc * n].view(n, ldc)[:, :m] for x in R)
    d = (C[0] - R[0]) + (C[1] - R[1])
    if not bool(torch.isfinite(d).all()):
        return float("inf")
    nr = float(torch.linalg.vector_norm(R[0]))
    return float(torch.linalg.vector_norm(d)) / nr / (k * 2.0 ** -104)


def bench_ozaki(h, args, stream, t_plain):
    """Split forms at n: for each kind and input set, the smallest slice count
    whose result agrees with the plain kernel's to <= 4 k 2^-104 (the plain
    result is itself within ~0.01 of the oracle on these inputs), then timed."""
    import torch
    import workloads as W
    from paper_2109_13406_amd import binding as b
    n = args.n
    out = {}
    for dist in ("uniform", "wide"):
        case = W.gemm_case_device(W.BASE_SEED + 3, "N", "N", n, n, n, dist=dist)
        C0 = tuple(x.clone() for x in case["C"])
        P = tuple(x.clone() for x in C0)
        args_ = ("N", "N", n, n, n, case["alpha"], case["A"], case["lda"], case["B"], case["ldb"],
                 case["beta"])
        assert b.mpdd_Rgemm(h, *args_, P, case["ldc"], stream=stream) == 0
        for kind, algo, rng_s in (("i8", b.MPDD_OZAKI_I8, range(13, 25)),
                                  ("f64", b.MPDD_OZAKI_F64, range(4, 11))):
            C = tuple(torch.empty_like(x) for x in C0)
            found = None
            for sl in rng_s:
                for dst, src in zip(C, C0):
                    dst.copy_(src)
                info = b.mpdd_Rgemm_ex(h, dict(algo=algo, nslices=sl), *args_, C, case["ldc"],
                                       stream=stream)
                if info != 0:
                    break
                r = ratio_gpu(C, P, n, n, case["ldc"], n)
                if r <= 4.0:
                    found = (sl, r)
                    break
            if found is None:
                out[f"{kind}_{dist}"] = {"nslices": None}
                continue
            sl, r = found

            def step():
                info = b.mpdd_Rgemm_ex(h, dict(algo=algo, nslices=sl), *args_, C, case["ldc"],
                                       stream=stream)
                if info != 0:
                    raise RuntimeError(info)
            _, per = timed_calls(step, 3, 1, stream)
            t = sum(per) / len(per)
            pairs = sl * (sl + 1) // 2
            rec = {"nslices": sl, "ratio_vs_plain": round(r, 4), "ms": round(t * 1e3, 2),
                   "dd_gflops": round(2.0 * n ** 3 / t / 1e9, 1),
                   "speedup_vs_plain": round(t_plain / t, 3),
                   "slice_products": pairs}
            if kind == "i8":
                rec["int8_tops_whole_call"] = round(pairs * 2.0 * n ** 3 / t / 1e12, 1)
                rec["int8_peak_tops"] = INT8_PEAK_TOPS
            else:
                rec["fp64_mfma_tflops_whole_call"] = round(pairs * 2.0 * n ** 3 / t / 1e12, 2)
                rec["fp64_peak_tflops"] = FP64_PEAK_TFLOPS
            out[f"{kind}_{dist}"] = rec
            log(f"ozaki {kind} {dist}: {rec}")
        del case, C0, P, C
        torch.cuda.empty_cache()
    return out


def bench_host(h, args):
    """MPBLAS-shaped host call (dd_real pairs in host memory) at n: copies to
    the device and back are inside the timed call, as in the manual's "with
    host-GPU transfer" figures."""
    import torch
    import workloads as W
    from paper_2109_13406_amd import binding as b
    n = args.n
    case = W.gemm_case_device(W.BASE_SEED + 5, "N", "N", n, n, n)
    hp = lambda pl: torch.stack([pl[0], pl[1]], dim=1).cpu().numpy()
    A, B, C = hp(case["A"]), hp(case["B"]), hp(case["C"])
    del case
    torch.cuda.empty_cache()
    ld = W.ld_padded(n)
    times = []
    for it in range(3):
        t0 = time.perf_counter()
        info = b.mpdd_Rgemm_host(h, "N", "N", n, n, n, (0.5, 0.0), A, ld, B, ld, (0.25, 0.0), C,
                                 ld)
        dt = time.perf_counter() - t0
        if info != 0:
            raise RuntimeError(f"mpdd_Rgemm_host info={info}")
        if it > 0:
            times.append(dt)
    t = min(times)
    return {"workload": f"Rgemm NN m=n=k={n} ld={ld}, dd_real pairs in pageable host memory",
            "ms": round(t * 1e3, 2), "dd_gflops_with_transfer": round(2.0 * n ** 3 / t / 1e9, 1),
            "host_bytes_moved": 16 * ld * n * 4}


def bench_serve(h, args):
    """Served request stream (Poisson arrivals) vs the same requests issued as
    sequential plain calls; p50 / p99 latency and aggregate dd-GFLOPS."""
    import torch
    import workloads as W
    from paper_2109_13406_amd.loadgen import Arena, percentiles, sequential, serve
    out = {}
    for rate, count in ((1000.0, args.serve_count), (100.0, args.serve_count_slow)):
        reqs = W.request_stream(W.BASE_SEED + 4, count, rate)
        arena = Arena(reqs, seed=W.BASE_SEED + 4)
        flops = sum(arena.flops(i) for i in range(count))
        arena.reset_c()
        tm, wall = serve(h, arena, paced=True)
        bad = sum(1 for t in tm if t["info"] != 0)
        lat = [t["end"] - t["arrival"] for t in tm]
        groups = len({t["group"] for t in tm})
        arena.reset_c()
        slat, swall = sequential(h, arena, paced=True)
        arena.reset_c()
        tb, bwall = serve(h, arena, paced=False)
        arena.reset_c()
        _, sbwall = sequential(h, arena, paced=False)
        rec = {"requests": count, "rate_per_s": rate, "failed": bad, "groups": groups,
               "served": {k: round(v * 1e3, 3) for k, v in percentiles(lat).items()},
               "sequential": {k: round(v * 1e3, 3) for k, v in percentiles(slat).items()},
               "latency_unit": "ms",
               "served_dd_gflops": round(flops / wall / 1e9, 1),
               "sequential_dd_gflops": round(flops / swall / 1e9, 1),
               "back_to_back_served_dd_gflops": round(flops / bwall / 1e9, 1),
               "back_to_back_sequential_dd_gflops": round(flops / sbwall / 1e9, 1),
               "offered_dd_gflops": round(flops / reqs[-1]["arrival"] / 1e9, 1)}
        out[f"poisson_{int(rate)}"] = rec
        log(f"serve {rate}/s: {rec}")
        del arena
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--sections", default="plain,sizes,syrk,cgemm,potrf,qd,ozaki,host,serve")
    ap.add_argument("--tile", type=int, default=-1,
                    help="tile-table entry for the plain product (-1: the library's choice)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="first run one device-to-device copy of BYTES bytes (a kernel of known "
                         "traffic, to calibrate the HBM byte counters of a profiling pass)")
    ap.add_argument("--serve-count", type=int, default=10000)
    ap.add_argument("--serve-count-slow", type=int, default=1000)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(each request / product runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2109_13406_amd import binding as b
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    h = b.mpdd_create()
    sections = set(args.sections.split(","))
    n = args.n
    if args.copy_probe:
        src = torch.empty(args.copy_probe // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe} bytes")
        del src, dst
        torch.cuda.empty_cache()

    case, total, per = bench_plain(h, args, stream)
    t_step = total / args.steps
    flops = 2.0 * n * n * n
    value = flops / t_step / 1e9
    t_kernel = sum(per) / len(per)
    madds = float(n) ** 3
    achieved = 2.0 * OPS_PER_MADD_ALG * madds / t_kernel / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 2), "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
            "traffic": traffic_record("dd_gemm_nn8192"),
            "kernel": "dd_gemm_kernel (plain, NN)",
            "kernel_ms": round(t_kernel * 1e3, 3),
            "issue_frac": round(OPS_PER_MADD_LEAN * madds / t_kernel / (FP64_PEAK_TFLOPS / 2 * 1e12), 4)}
    log(f"plain NN {n}: {t_step*1e3:.2f} ms/step, {value:.1f} dd-GFLOPS, kernel {t_kernel*1e3:.2f} ms")

    out = {"metric": METRIC, "value": round(value, 1), "unit": "dd-GFLOPS", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t_step * 1e3, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"Rgemm NN m=n=k={n} lda=ldb=ldc={case['lda']} dd "
                                  "(float64 hi/lo planes, hi~U[-1,1), plain form)",
                      "m": n, "n": n, "k": n, "algo": "plain"},
           "roofline": roof}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(case, n)
        log(f"cpu baseline: {out['cpu_baseline']}")
    del case
    torch.cuda.empty_cache()
    if "syrk" in sections:
        out["rsyrk"] = bench_syrk(h, args, stream)
        log(f"rsyrk: {out['rsyrk']}")
    if "sizes" in sections:
        out["rgemm_sizes"] = bench_sizes(h, args, stream)
    if "qd" in sections:
        out["qgemm"] = bench_qd(h, args, stream)
        log(f"qgemm: {out['qgemm']}")
    if "potrf" in sections:
        out["rpotrf"] = bench_potrf(h, args, stream)
        log(f"rpotrf: {out['rpotrf']}")
    if "cgemm" in sections:
        out["cgemm"] = bench_cgemm(h, args, stream)
        log(f"cgemm: {out['cgemm']}")
    if "ozaki" in sections:
        out["ozaki"] = bench_ozaki(h, args, stream, t_kernel)
    if "host" in sections:
        out["host_api"] = bench_host(h, args)
        log(f"host api: {out['host_api']}")
    if "serve" in sections:
        out["serving"] = bench_serve(h, args)
    out["context"] = {"paper_dd_rgemm_gflops": {"A100": 592, "V100": 435},
                      "paper_dd_rsyrk_gflops": {"V100": 428},
                      "paper_dd_rgemm_gflops_with_transfer": {"V100": 318},
                      "dd_roofline_tflops": round(2 * FP64_PEAK_TFLOPS / 2 / OPS_PER_MADD_ALG, 3)}
    torch.cuda.synchronize()
    b.mpdd_destroy(h)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
