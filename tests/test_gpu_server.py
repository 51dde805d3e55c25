"""The request server on the GPU: every served result is bit-identical to the
same request run alone through the server and to a standalone call with the
same tile, and within 8 k 2^-104 of the oracle; a tight memory budget still
completes every request."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import log
from oracle.compare import RATIO_MAX, bits, ratio

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import torch
    from paper_2109_13406_amd import binding as b
    handle = b.mpdd_create()
    yield handle
    torch.cuda.synchronize()
    b.mpdd_destroy(handle)


@pytest.fixture(scope="module")
def arena():
    from paper_2109_13406_amd.loadgen import Arena
    reqs = W.request_stream(4242, 120, rate=1000.0, lo=16, hi=300)
    return Arena(reqs, seed=77)


def _c_region(arena, i):
    r = arena.reqs[i]
    m = r["m"] if r["kind"] == "gemm" else r["n"]
    off = arena.c_off[i]
    return tuple(x[off: off + m * r["n"]].cpu().numpy() for x in arena.c)


def _snapshot(arena):
    import torch
    torch.cuda.synchronize()
    return [_c_region(arena, i) for i in range(len(arena.reqs))]


def _same(a, b_, i, what):
    assert np.array_equal(bits(a[0]), bits(b_[0])) and np.array_equal(bits(a[1]), bits(b_[1])), \
        f"request {i}: {what}"


def test_served_mix_equals_alone_and_standalone(h, arena):
    import torch
    from paper_2109_13406_amd import binding as b
    from paper_2109_13406_amd.loadgen import serve
    arena.reset_c()
    timings, _ = serve(h, arena, paced=False)
    assert all(t["info"] == 0 for t in timings)
    mix = _snapshot(arena)
    groups = {t["group"] for t in timings}
    log(f"SERVE mix: {len(arena.reqs)} requests in {len(groups)} groups")

    # each request alone through the server
    arena.reset_c()
    s = b.mpdd_server_create(h, 1 << 36, 64)
    for i in range(len(arena.reqs)):
        t = b.mpdd_server_submit(s, arena.request(i))
        info, tm = b.mpdd_server_wait(s, t)
        assert info == 0
        assert tm["tile"] == timings[i]["tile"]
    b.mpdd_server_destroy(s)
    alone = _snapshot(arena)

    # each request as a standalone call with the served tile
    arena.reset_c()
    stream = torch.cuda.current_stream()
    for i in range(len(arena.reqs)):
        assert arena.call_plain(h, i, stream, tile_id=timings[i]["tile"]) == 0
    plain = _snapshot(arena)
    for i in range(len(arena.reqs)):
        _same(mix[i], alone[i], i, "mix vs alone")
        _same(mix[i], plain[i], i, "served vs standalone call")
    log("SERVE results bit-identical: mix == alone == standalone call")


def test_served_results_match_oracle(h, arena):
    from paper_2109_13406_amd.loadgen import serve
    arena.reset_c()
    c0 = _snapshot(arena)
    timings, _ = serve(h, arena, paced=False)
    got = _snapshot(arena)
    worst = 0.0
    for i in range(0, len(arena.reqs), 4):
        r = arena.reqs[i]
        A, lda, B, ldb, C, ldc = arena.ptrs(i)
        alpha, beta = arena.scal[i]
        ao, bo = arena.a_off[i], arena.b_off[i]
        if r["kind"] == "gemm":
            m, n, k = r["m"], r["n"], r["k"]
            na = lda * (k if r["transa"] == "N" else m)
            nb = ldb * (n if r["transb"] == "N" else k)
            Ah = tuple(x[ao: ao + na].cpu().numpy() for x in arena.ab)
            Bh = tuple(x[bo: bo + nb].cpu().numpy() for x in arena.ab)
            O = (c0[i][0].copy(), c0[i][1].copy())
            assert oracle.rgemm(r["transa"], r["transb"], m, n, k, alpha, Ah, lda, Bh, ldb, beta,
                                O, ldc) == 0
            rr = ratio(got[i][0], got[i][1], O[0], O[1], k)
        else:
            n, k = r["n"], r["k"]
            na = lda * (k if r["trans"] == "N" else n)
            Ah = tuple(x[ao: ao + na].cpu().numpy() for x in arena.ab)
            O = (c0[i][0].copy(), c0[i][1].copy())
            assert oracle.rsyrk(r["uplo"], r["trans"], n, k, alpha, Ah, lda, beta, O, ldc) == 0
            ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
            sel = (ii <= jj) if r["uplo"] == "U" else (ii >= jj)
            idx = (ii + jj * n)[sel]
            rr = ratio(got[i][0][idx], got[i][1][idx], O[0][idx], O[1][idx], k)
            rest = (ii + jj * n)[~sel]
            assert np.array_equal(bits(got[i][0][rest]), bits(c0[i][0][rest]))
        worst = max(worst, rr)
        assert rr <= RATIO_MAX, (i, r, rr)
    log(f"SERVE results vs oracle: worst ratio {worst:.3g}")


def test_tight_budget_completes_everything(h, arena):
    from paper_2109_13406_amd import binding as b
    arena.reset_c()
    sizes = []
    for i in range(len(arena.reqs)):
        r = arena.request(i)
        sizes.append(r)
    one = max(16 * (r.lda * max(r.k, r.m, r.n) + r.ldb * max(r.n, r.k) + r.ldc * r.n)
              for r in sizes)
    s = b.mpdd_server_create(h, 3 * one, 1 << 20)
    tickets = [b.mpdd_server_submit(s, q) for q in sizes]
    tms = [b.mpdd_server_wait(s, t) for t in tickets]
    b.mpdd_server_destroy(s)
    assert all(info == 0 for info, _ in tms)
    admits = [tm["admit"] for _, tm in tms]
    assert admits == sorted(admits)


def test_served_stream_verified_like_the_benchmark(h, arena):
    """The benchmark's check of a served stream (every request, sampled
    entries against the oracle) on this stream: all within 8 k 2^-104."""
    import bench
    from paper_2109_13406_amd.loadgen import serve
    arena.reset_c()
    timings, _ = serve(h, arena, paced=False)
    assert all(t["info"] == 0 for t in timings)
    check = bench.verify_served(arena, samples=8, seed=99)
    log(f"SERVE verify_served: {check}")
    assert check["requests"] == len(arena.reqs)
    assert check["over_tolerance"] == 0 and check["worst_ratio"] <= RATIO_MAX


def test_tuned_table_picks_served_tiles(arena, tmp_path):
    """A tile table written by the autotuner steers the server: with the
    32 x 32 tile recorded as the served tile of every bucket, every request
    runs with it, and each result is bit-identical to a standalone call with
    that tile.  A malformed table is refused at handle creation."""
    import torch
    from paper_2109_13406_amd import autotune as AT
    from paper_2109_13406_amd import binding as b
    from paper_2109_13406_amd.loadgen import serve
    entries = []
    for op, combos in (("gemm", ("NN", "NT", "TN", "TT")), ("syrk", ("NT", "TN"))):
        for mb in range(0, 10):
            for nb in range(0, 10):
                for kb in range(0, 10):
                    if op == "syrk" and mb != nb:
                        continue
                    for tr in combos:
                        entries.append(dict(op=op, trans=tr, mb=mb, nb=nb, kb=kb, tile=4,
                                            splitk=1, serve_tile=2, dd_gflops=0.0))
    path = str(tmp_path / "tune.json")
    AT.write_cache(path, entries)
    ht = b.mpdd_create(path)
    try:
        arena.reset_c()
        timings, _ = serve(ht, arena, paced=False)
        assert all(t["info"] == 0 and t["tile"] == 2 for t in timings)
        served = _snapshot(arena)
        arena.reset_c()
        stream = torch.cuda.current_stream()
        for i in range(len(arena.reqs)):
            assert arena.call_plain(ht, i, stream, tile_id=2) == 0
        plain = _snapshot(arena)
        for i in range(len(arena.reqs)):
            _same(served[i], plain[i], i, "tuned served tile vs standalone call")
    finally:
        torch.cuda.synchronize()
        b.mpdd_destroy(ht)
    bad = tmp_path / "bad.json"
    bad.write_text('{"entries": [\n{"op": "gemm", "trans": "NN", "mb": 1}\n]}\n')
    with pytest.raises(RuntimeError):
        b.mpdd_create(str(bad))
    log("SERVE tuned table: served tiles follow the table")
