// tuner.cpp -- the tuning table of a handle (see tuner.hpp).
#include "tuner.hpp"

#include <algorithm>
#include <cstdio>
#include <cstring>

#include "kernels.hpp"

namespace mpdd {

int shape_bucket(int64_t x) {
  int b = 0;
  while (b < 62 && ((int64_t)1 << b) < x) ++b;
  return b;
}

static int op_code(const char* s) {
  if (std::strcmp(s, "gemm") == 0) return 0;
  if (std::strcmp(s, "syrk") == 0) return 1;
  return -1;
}

bool TuneTable::load(const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool ok = true;
  while (std::fgets(line, sizeof line, f)) {
    const char* p = std::strstr(line, "{\"op\"");
    if (!p) continue;
    char op[8] = {0}, tr[4] = {0};
    int mb, nb, kb, tile, splitk, nsl = 0;
    int got = std::sscanf(p,
                          "{\"op\": \"%7[a-z]\", \"trans\": \"%3[NT]\", \"mb\": %d, \"nb\": %d, "
                          "\"kb\": %d, \"tile\": %d, \"splitk\": %d, \"nslices\": %d",
                          op, tr, &mb, &nb, &kb, &tile, &splitk, &nsl);
    const int code = op_code(op);
    if (got < 7 || code < 0 || std::strlen(tr) != 2 || !tile_info(tile) || splitk < 1) {
      ok = false;
      break;
    }
    TuneEntry e;
    e.tile = tile;
    e.splitk = splitk;
    e.nslices = nsl;
    if (const char* st = std::strstr(p, "\"serve_tile\":")) {
      int t = -1;
      if (std::sscanf(st, "\"serve_tile\": %d", &t) != 1 || (t >= 0 && !tile_info(t))) {
        ok = false;
        break;
      }
      e.serve_tile = t;
    }
    map_[Key(code, tr[0] == 'T', tr[1] == 'T', mb, nb, kb)] = e;
  }
  std::fclose(f);
  return ok;
}

bool TuneTable::lookup(int op, bool ta, bool tb, int64_t m, int64_t n, int64_t k,
                       TuneEntry& out) const {
  auto it = map_.find(Key(op, ta, tb, shape_bucket(m), shape_bucket(n), shape_bucket(k)));
  if (it == map_.end()) return false;
  out = it->second;
  return true;
}

// 64 x 64 tiles with the cross terms on the matrix cores (entry 4) when,
// split along k into ranges of >= 512, they give enough workgroups (512;
// 1024 for a triangle); otherwise 32 x 32 tiles (entry 2), four times the
// workgroups.  Measured on skinny and small shapes (the block-column updates
// of Rpotrf: 2048 x 64 x 6080 NT 657 -> 329 us, 7936 x 64 x 192 117 -> 53 us;
// Rsyrk 2048 x 512: 533 -> 441 us) with no loss on the large ones.  Both
// entries are square, so the choice also serves triangles and served groups.
int default_tile(int64_t m, int64_t n, int64_t k, bool tri) {
  const int64_t tm = (m + 63) / 64, tn = (n + 63) / 64;
  const int64_t tiles = tri ? tm * (tm + 1) / 2 : tm * tn;
  const int64_t smax = std::min<int64_t>(32, std::max<int64_t>(1, k / 512));
  return tiles * smax < (tri ? 1024 : 512) ? 2 : 4;
}

}  // namespace mpdd
