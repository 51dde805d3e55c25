"""Load generator for the request server: builds device-resident operands for
a stream of Rgemm / Rsyrk requests, submits them at their (Poisson) arrival
times, and collects per-request timings -- or issues the same requests as
sequential plain calls for comparison.

Operands: A and B of every request are read-only views into one shared
random dd "arena" (so 10,000 requests do not need 10,000 fresh matrices),
each request gets its own C region (written), leading dimensions = rows.
"""
import math
import time

import numpy as np

from . import binding as b


class Arena:
    """Device buffers for a request list.  `reqs`: dicts from
    workloads.request_stream (kind, flags, m, n, k, ...)."""

    def __init__(self, reqs, seed=20264, device="cuda", random_c=None):
        import torch
        import workloads as W
        self.reqs = reqs
        need_ab = 0
        for r in reqs:
            if r["kind"] == "gemm":
                need_ab = max(need_ab, r["m"] * r["k"], r["k"] * r["n"])
            else:
                need_ab = max(need_ab, r["n"] * r["k"])
        size = max(1 << 22, 2 * need_ab)
        self.ab = W.dd_matrix_device(seed, size, 1, size, "uniform", device)
        rng = np.random.default_rng(seed)
        self.c_off = []
        total = 0
        for r in reqs:
            m = r["m"] if r["kind"] == "gemm" else r["n"]
            self.c_off.append(total)
            total += m * r["n"]
        self.c_total = total
        self.c = tuple(torch.empty(max(1, total), dtype=torch.float64, device=device)
                       for _ in range(2))
        if random_c is None:
            random_c = total <= (1 << 27)
        if random_c:
            self.c0 = W.dd_matrix_device(seed + 1, max(1, total), 1, max(1, total), "uniform",
                                         device)
        else:   # very long streams: C starts at zero (beta * 0)
            self.c0 = tuple(torch.zeros(max(1, total), dtype=torch.float64, device=device)
                            for _ in range(2))
        self.a_off, self.b_off = [], []
        for r in reqs:
            if r["kind"] == "gemm":
                na, nb = r["m"] * r["k"], r["k"] * r["n"]
            else:
                na, nb = r["n"] * r["k"], 0
            self.a_off.append(int(rng.integers(0, size - na + 1)))
            self.b_off.append(int(rng.integers(0, size - nb + 1)))
        self.scal = []
        for i, _ in enumerate(reqs):
            ra = np.random.default_rng(seed * 7 + i)
            self.scal.append(((float(ra.uniform(-1, 1)), 0.0), (float(ra.uniform(-1, 1)), 0.0)))
        torch.cuda.synchronize()

    def reset_c(self):
        for dst, src in zip(self.c, self.c0):
            dst.copy_(src)

    def ptrs(self, i):
        """(A, lda, B, ldb, C, ldc) device pointers of request i."""
        r = self.reqs[i]
        esz = 8
        ah = self.ab[0].data_ptr() + esz * self.a_off[i]
        al = self.ab[1].data_ptr() + esz * self.a_off[i]
        bh = self.ab[0].data_ptr() + esz * self.b_off[i]
        bl = self.ab[1].data_ptr() + esz * self.b_off[i]
        ch = self.c[0].data_ptr() + esz * self.c_off[i]
        cl = self.c[1].data_ptr() + esz * self.c_off[i]
        if r["kind"] == "gemm":
            lda = r["m"] if r["transa"] == "N" else r["k"]
            ldb = r["k"] if r["transb"] == "N" else r["n"]
            ldc = r["m"]
        else:
            lda = r["n"] if r["trans"] == "N" else r["k"]
            ldb = 1
            ldc = r["n"]
        return (ah, al), lda, (bh, bl), ldb, (ch, cl), ldc

    def request(self, i, arrival=-1.0):
        r = self.reqs[i]
        A, lda, B, ldb, C, ldc = self.ptrs(i)
        alpha, beta = self.scal[i]
        if r["kind"] == "gemm":
            return b.make_request(b.MPDD_OP_GEMM, r["transa"], r["transb"], r["m"], r["n"],
                                  r["k"], alpha, A, lda, B, ldb, beta, C, ldc, arrival=arrival)
        return b.make_request(b.MPDD_OP_SYRK, r["uplo"], r["trans"], 0, r["n"], r["k"], alpha,
                              A, lda, (None, None), 1, beta, C, ldc, arrival=arrival)

    def call_plain(self, h, i, stream, tile_id=-1):
        """The same request as one plain library call (default or given tile)."""
        r = self.reqs[i]
        A, lda, B, ldb, C, ldc = self.ptrs(i)
        alpha, beta = self.scal[i]
        opts = dict(algo=b.MPDD_PLAIN, tile_id=tile_id, splitk=1 if tile_id >= 0 else 0)
        if r["kind"] == "gemm":
            return b.mpdd_Rgemm_ex(h, opts, r["transa"], r["transb"], r["m"], r["n"], r["k"],
                                   alpha, A, lda, B, ldb, beta, C, ldc, stream=stream)
        return b.mpdd_Rsyrk_ex(h, opts, r["uplo"], r["trans"], r["n"], r["k"], alpha, A, lda,
                               beta, C, ldc, stream=stream)

    def prepared_plain(self, h, i, stream):
        """call_plain with its arguments marshalled now: a callable issuing
        the call (returns info)."""
        r = self.reqs[i]
        A, lda, B, ldb, C, ldc = self.ptrs(i)
        alpha, beta = self.scal[i]
        opts = dict(algo=b.MPDD_PLAIN, tile_id=-1, splitk=0)
        if r["kind"] == "gemm":
            return b.prepared_Rgemm_ex(h, opts, r["transa"], r["transb"], r["m"], r["n"], r["k"],
                                       alpha, A, lda, B, ldb, beta, C, ldc, stream=stream)
        return b.prepared_Rsyrk_ex(h, opts, r["uplo"], r["trans"], r["n"], r["k"], alpha, A, lda,
                                   beta, C, ldc, stream=stream)

    def flops(self, i):
        r = self.reqs[i]
        if r["kind"] == "gemm":
            return 2.0 * r["m"] * r["n"] * r["k"]
        return float(r["n"]) * (r["n"] + 1) * r["k"]


def _pace(clock, arr):
    while clock() < arr:
        d = arr - clock()
        if d > 2e-3:
            time.sleep(d - 1e-3)


def serve(h, arena, budget=200 * 10 ** 9, max_inflight=4096, paced=True, progress=None):
    """Submit every request at its arrival time (paced) or all at once;
    returns (timings list, wall seconds).  Latency = end - arrival.  The
    request descriptors are built before the clock starts (as a client holds
    its work ready), so a request's latency counts the server, not the
    descriptor marshalling.  progress(i) is called every 2000 submissions."""
    s = b.mpdd_server_create(h, budget, max_inflight)
    try:
        n = len(arena.reqs)
        tickets = [0] * n
        reqs = [arena.request(i) for i in range(n)]
        submit = b.prepared_submit(s)
        clock = b.load().mpdd_clock
        t0 = clock() + 0.01
        for i, r in enumerate(arena.reqs):
            arr = t0 + (r["arrival"] if paced else 0.0)
            if paced:
                _pace(clock, arr)
            reqs[i].arrival = arr
            tickets[i] = submit(reqs[i])
            if progress is not None and i % 2000 == 1999:
                progress(i + 1)
        out = []
        for t in tickets:
            info, tm = b.mpdd_server_wait(s, t)
            tm["info"] = info
            out.append(tm)
        wall = max(tm["end"] for tm in out) - t0
    finally:
        b.mpdd_server_destroy(s)
    return out, wall


def sequential(h, arena, paced=True, progress=None):
    """The same requests as single plain calls on one stream in arrival order,
    each synchronised; paced = open loop with the same arrival times.  The
    calls' arguments are marshalled before the clock starts, as for serve().
    Returns (latencies, wall seconds)."""
    import torch
    stream = torch.cuda.current_stream()
    calls = [arena.prepared_plain(h, i, stream) for i in range(len(arena.reqs))]
    lat = []
    clock = time.perf_counter
    t0 = clock() + 0.01
    for i, r in enumerate(arena.reqs):
        arr = t0 + (r["arrival"] if paced else 0.0)
        if paced:
            _pace(clock, arr)
        info = calls[i]()
        if info != 0:
            raise RuntimeError(f"request {i}: info {info}")
        stream.synchronize()
        lat.append(clock() - arr)
        if progress is not None and i % 2000 == 1999:
            progress(i + 1)
    wall = clock() - t0
    return lat, wall


def percentiles(xs, ps=(50, 99)):
    a = np.sort(np.asarray(xs))
    return {f"p{p}": float(a[min(len(a) - 1, int(math.ceil(p / 100.0 * len(a))) - 1)]) for p in ps}
