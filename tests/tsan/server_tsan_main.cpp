// server_tsan_main.cpp -- drives the request server's host logic (fake-device
// mode: no GPU calls) from several threads, built with ThreadSanitizer by
// tests/test_server_tsan.py.  The kernel-launch and tile-table symbols that
// server.cpp references are stubbed here; the fake device never launches.
#include <atomic>
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include "../../include/mpdd.h"
#include "../../include/mpdd_testing.h"
#include "../../paper_2109_13406_amd/csrc/kernels.hpp"
#include "../../paper_2109_13406_amd/csrc/tuner.hpp"

namespace mpdd {
static const TileInfo kStubTiles[] = {{64, 64, 16, 256}, {64, 64, 8, 256}, {32, 32, 16, 256}};
int tile_count() { return 3; }
const TileInfo* tile_info(int id) { return (id >= 0 && id < 3) ? &kStubTiles[id] : nullptr; }
int default_tile(int64_t m, int64_t n, int64_t, bool) {
  return ((m + 63) / 64) * ((n + 63) / 64) < 128 ? 2 : 0;
}
hipError_t launch_grouped_list(int, const char*, const ServeReq*, const int*, const int*, int, int,
                               hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_gemm(int, const GemmParams&, bool, bool, bool, int, hipStream_t) {
  return hipErrorInvalidValue;
}
}  // namespace mpdd
bool handle_valid(const mpdd_handle_s*) { return false; }
int handle_device(const mpdd_handle_s*) { return 0; }
bool handle_tune_lookup(const mpdd_handle_s*, int, bool, bool, int64_t, int64_t, int64_t,
                        mpdd::TuneEntry&) {
  return false;
}

static mpdd_request gemm(int m, int n, int k, int inject) {
  mpdd_request r;
  std::memset(&r, 0, sizeof r);
  r.op = MPDD_OP_GEMM;
  r.flag1 = 'N';
  r.flag2 = 'N';
  r.m = m; r.n = n; r.k = k;
  r.alpha.hi = 1.0; r.beta.hi = 0.5;
  const double* P = (const double*)0x1000;
  r.A_hi = r.A_lo = P; r.lda = m;
  r.B_hi = r.B_lo = P; r.ldb = k;
  r.C_hi = r.C_lo = (double*)0x1000; r.ldc = m;
  r.arrival = -1.0;
  r.inject = inject;
  return r;
}

int main() {
  mpdd_server s = nullptr;
  const size_t one = 16 * (size_t)(64 * 64 * 3);
  if (mpdd_server_create(&s, nullptr, 6 * one, 64, MPDD_SERVER_FAKE_DEVICE) != 0) return 2;
  mpdd_server_set_fake_rate(s, 1e9, 50e-6);
  std::atomic<int> bad{0}, done{0};
  std::vector<std::thread> th;
  for (int t = 0; t < 6; ++t)
    th.emplace_back([&] {
      std::vector<uint64_t> tickets;
      for (int i = 0; i < 60; ++i) {
        uint64_t tk;
        const int inject = (i % 17 == 5) ? MPDD_INJECT_DEVICE_ERROR : 0;
        const mpdd_request r = gemm(64, 64, 64, inject);
        if (mpdd_server_submit(s, &r, &tk) != 0) {
          bad++;
          continue;
        }
        tickets.push_back(tk);
        if (i % 7 == 0) {
          mpdd_server_stats st;
          mpdd_server_get_stats(s, &st);
          int d;
          mpdd_server_poll(s, tk, &d);
        }
      }
      for (size_t i = 0; i < tickets.size(); ++i) {
        int info;
        mpdd_timing tm;
        if (mpdd_server_wait(s, tickets[i], &info, &tm) != 0) bad++;
        const bool injected = (i % 17 == 5);
        if (injected ? info != MPDD_ERR_HIP : info != 0) bad++;
        done++;
      }
    });
  for (auto& x : th) x.join();
  // leave a few requests queued: destroy must drain them
  for (int i = 0; i < 10; ++i) {
    uint64_t tk;
    mpdd_request r = gemm(32, 32, 32, 0);
    mpdd_server_submit(s, &r, &tk);
  }
  mpdd_server_destroy(s);
  std::printf("done=%d bad=%d\n", done.load(), bad.load());
  return bad.load() == 0 && done.load() == 360 ? 0 : 1;
}
