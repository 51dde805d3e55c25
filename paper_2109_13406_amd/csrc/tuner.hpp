// tuner.hpp -- tile / k-split choice per (operation, flags, shape bucket).
// The table is filled by the autotuner (paper_2109_13406_amd/autotune.py),
// which times every candidate on the device and writes a JSON cache; the
// handle loads it at creation.  Without an entry, default_tile() applies.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>

namespace mpdd {

struct TuneEntry {
  int tile = -1;         // stand-alone calls: tile-table entry
  int splitk = 0;        // stand-alone calls: k-split
  int nslices = 0;
  int serve_tile = -1;   // request server (unsplit grouped launches): tile entry, -1 = tile
};

// Shape bucket: ceil(log2(x)) (0 for x <= 1).
int shape_bucket(int64_t x);

class TuneTable {
 public:
  // Reads the autotuner's JSON cache (one entry object per line).  Returns
  // false when the file cannot be read or an entry line is malformed.
  bool load(const char* path);
  bool lookup(int op, bool ta, bool tb, int64_t m, int64_t n, int64_t k, TuneEntry& out) const;
  size_t size() const { return map_.size(); }

 private:
  using Key = std::tuple<int, int, int, int, int, int>;
  std::map<Key, TuneEntry> map_;
};

// Built-in choice from the tile table when the tuner has no entry (tri: the
// product is a triangle, of which only the tiles meeting it are computed).
int default_tile(int64_t m, int64_t n, int64_t k, bool tri);

}  // namespace mpdd

struct mpdd_handle_s;

namespace mpdd { class HostStager; }
// The pinned staging of the host-pointer calls (host_api.cpp), owned by the
// handle: its lock, its stager slot, and its destruction with the handle.
std::mutex* handle_host_mutex(mpdd_handle_s* h);
// The handle's stream-ordered scratch pool.
hipMemPool_t handle_pool(const mpdd_handle_s* h);
// which = 0: the stager of copies to the device, 1: of copies back
mpdd::HostStager** handle_stager(mpdd_handle_s* h, int which);
void destroy_stager(mpdd::HostStager* st);
// Handle accessors for other translation units (mpdd.cpp owns the struct).
bool handle_valid(const mpdd_handle_s* h);
int handle_device(const mpdd_handle_s* h);
bool handle_tune_lookup(const mpdd_handle_s* h, int op, bool ta, bool tb, int64_t m, int64_t n,
                        int64_t k, mpdd::TuneEntry& out);
