"""Autotuner for the plain dd kernels: times every (tile, k-split) candidate
on the device for a set of shapes and writes the JSON cache that
mpdd_create(h, path) loads.

    python -m paper_2109_13406_amd.autotune --out tune.json [--shapes serve|bench|all]

Shapes are bucketed by ceil(log2) of m, n, k (the library looks entries up by
bucket), so one timed representative per bucket covers the bucket.  Each
candidate is run once to warm up and then timed over `reps` calls with HIP
events; inputs are seeded uniform dd matrices resident in HBM.
"""
import argparse
import json
import math
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def bucket(x):
    return max(0, math.ceil(math.log2(max(1, x))))


def _time(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / 1e3 / reps


def tune_shape(h, op, ta, tb, m, n, k, reps=3, splits=(1, 2, 4, 8, 16), verbose=True):
    """Best (tile, splitk, seconds) for one shape, and every timing."""
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import workloads as W
    from paper_2109_13406_amd import binding as b
    results = []
    if op == "gemm":
        case = W.gemm_case_device(1234, ta, tb, m, n, k, padded=False)
    else:
        case = W.syrk_case_device(1234, "U", "N", n, k, padded=False)
    for tile in range(b.mpdd_tile_count()):
        bm, bn, bk, _ = b.mpdd_tile_info(tile)
        if op == "syrk" and bm != bn:
            continue
        for s in splits:
            if s > 1 and (k // s < 2 * bk):
                continue
            opts = dict(algo=b.MPDD_PLAIN, tile_id=tile, splitk=s)
            if op == "gemm":
                fn = lambda: b.mpdd_Rgemm_ex(h, opts, ta, tb, m, n, k, case["alpha"], case["A"],
                                             case["lda"], case["B"], case["ldb"], case["beta"],
                                             case["C"], case["ldc"])
            else:
                fn = lambda: b.mpdd_Rsyrk_ex(h, opts, "U", "N", n, k, case["alpha"],
                                             case["A"], case["lda"], case["beta"], case["C"],
                                             case["ldc"])
            info = fn()
            if info != 0:
                continue
            t = _time(fn, reps)
            flops = 2.0 * m * n * k if op == "gemm" else float(n) * (n + 1) * k
            results.append(dict(tile=tile, splitk=s, seconds=t, dd_gflops=flops / t / 1e9))
            if verbose:
                print(f"  {op} {ta}{tb} {m}x{n}x{k} tile {tile} ({bm}x{bn}x{bk}) split {s}: "
                      f"{t*1e3:.3f} ms {flops/t/1e9:.1f} dd-GFLOPS", flush=True)
    best = min(results, key=lambda r: r["seconds"])
    return best, results


SERVE_TILES = (2, 4)   # tile entries the request server's grouped launches run (unsplit)


def serve_best(results):
    """Fastest unsplit candidate among the tiles the server runs (None if
    none was timed)."""
    cand = [r for r in results if r["splitk"] == 1 and r["tile"] in SERVE_TILES]
    return min(cand, key=lambda r: r["seconds"]) if cand else None


def tune_ozaki(h, n, kind="i8", slices=(13, 16), reps=2, verbose=True):
    """Time the split form's product-kernel variants (tile_id) at m = n = k."""
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import workloads as W
    from paper_2109_13406_amd import binding as b
    algo = b.MPDD_OZAKI_I8 if kind == "i8" else b.MPDD_OZAKI_F64
    case = W.gemm_case_device(4321, "N", "N", n, n, n, padded=False)
    out = []
    for var in range(8 if kind == "i8" else 1):
        for sl in slices:
            opts = dict(algo=algo, nslices=sl, tile_id=var)
            fn = lambda: b.mpdd_Rgemm_ex(h, opts, "N", "N", n, n, n, case["alpha"], case["A"],
                                         case["lda"], case["B"], case["ldb"], case["beta"],
                                         case["C"], case["ldc"])
            if fn() != 0:
                continue
            t = _time(fn, reps)
            out.append(dict(variant=var, nslices=sl, seconds=t, dd_gflops=2.0 * n ** 3 / t / 1e9,
                            int8_tops=sl * (sl + 1) / 2 * 2.0 * n ** 3 / t / 1e12))
            if verbose:
                print(f"  ozaki {kind} n={n} variant {var} s={sl}: {t*1e3:.2f} ms "
                      f"{out[-1]['int8_tops']:.0f} T(int)ops/s", flush=True)
    return out


SHAPE_SETS = {
    "bench": [("gemm", "N", "N", 8192, 8192, 8192), ("gemm", "N", "N", 4096, 4096, 4096),
              ("gemm", "N", "N", 8192, 64, 8192), ("gemm", "N", "N", 4096, 4096, 256),
              ("syrk", "N", "N", 8192, 8192, 8192), ("syrk", "N", "N", 2048, 2048, 512)],
}


def serve_shapes():
    """One representative per (op, bucket) over log-uniform sizes 32..2048."""
    reps = [48, 96, 192, 384, 768, 1536]
    out = []
    for m in reps:
        for n in reps:
            for k in reps:
                out.append(("gemm", "N", "N", m, n, k))
    for n in reps:
        for k in reps:
            out.append(("syrk", "N", "N", n, n, k))
    return out


def write_cache(path, entries):
    """One entry object per line: op, flags, shape buckets, the stand-alone
    (tile, splitk) and, for the request server, the best unsplit served tile."""
    with open(path, "w") as f:
        f.write('{"version": 1, "arch": "gfx950", "entries": [\n')
        lines = []
        for e in entries:
            lines.append('{"op": "%s", "trans": "%s", "mb": %d, "nb": %d, "kb": %d, "tile": %d, '
                         '"splitk": %d, "nslices": 0, "serve_tile": %d, "dd_gflops": %.1f}'
                         % (e["op"], e["trans"], e["mb"], e["nb"], e["kb"], e["tile"],
                            e["splitk"], e.get("serve_tile", -1), e["dd_gflops"]))
        f.write(",\n".join(lines))
        f.write("\n]}\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--shapes", default="bench")
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import torch
    from paper_2109_13406_amd import binding as b
    h = b.mpdd_create()
    if args.shapes == "ozaki":
        rep = {n: tune_ozaki(h, n) for n in (4096, 8192)}
        with open(args.out, "w") as f:
            json.dump(rep, f, indent=1)
        b.mpdd_destroy(h)
        return
    shapes = serve_shapes() if args.shapes == "serve" else SHAPE_SETS[args.shapes]
    entries, report = [], []
    for (op, ta, tb, m, n, k) in shapes:
        best, res = tune_shape(h, op, ta, tb, m, n, k, reps=args.reps)
        print(f"BEST {op} {ta}{tb} {m}x{n}x{k}: tile {best['tile']} split {best['splitk']} "
              f"{best['dd_gflops']:.1f} dd-GFLOPS", flush=True)
        sb = serve_best(res)
        combos = ("NN", "NT", "TN", "TT") if op == "gemm" else ("NT", "TN")
        for tr in combos:
            entries.append(dict(op=op, trans=tr, mb=bucket(m), nb=bucket(n), kb=bucket(k),
                                tile=best["tile"], splitk=best["splitk"],
                                serve_tile=sb["tile"] if sb else -1,
                                dd_gflops=best["dd_gflops"]))
        report.append(dict(op=op, m=m, n=n, k=k, best=best, all=res))
        torch.cuda.empty_cache()
    write_cache(args.out, entries)
    with open(args.out + ".report.json", "w") as f:
        json.dump(report, f, indent=1)
    torch.cuda.synchronize()
    b.mpdd_destroy(h)


if __name__ == "__main__":
    main()
