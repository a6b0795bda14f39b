// tune.hip -- choice of the streaming-kernel tile (rows per thread) of each
// bisection level.
//
// The tile sets how many rows one workgroup of the SpMV/projection and
// update kernels covers (256 * rpt) and therefore also how many per-block
// partial sums the segmented reductions add up.  The built-in rule takes 4
// rows per thread.  The tuner instead times one Lanczos step of the level
// (both streaming launches and their reductions) for every candidate tile
// and keeps the fastest; results are kept per process and, when a cache file
// is named, in that file as one line per problem class:
//
//   rsb-tile 2 <gfx arch> <precision> <log2 rows> <nonzeros per row> <log2 segments> <m>
//              <steps per launch sequence: 1, or 2 for the two-step form> <rpt>
//
// A class is the level's size, density and segment count rounded as above,
// so one tuned entry serves every level and mesh of similar shape.  The
// reduction order follows the tile, so results are reproducible for a fixed
// tile (a fixed cache) but may differ in the last bits between tiles.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>

#include "common.h"
#include "kernels.h"

namespace rsb {

namespace {

constexpr int kCandidates[] = {2, 4, 8};

using TileKey = std::string;  // "<arch> <precision> <log2 rows> <nnz/row> <log2 segs> <m> <s>"

std::mutex g_tune_mu;
std::map<TileKey, int> g_tiles;              // tuned in this process or read from files
std::map<std::string, bool> g_files_read;    // cache files already merged into g_tiles

int ilog2(int64_t v) {
  int r = 0;
  while (v > 1) {
    v >>= 1;
    ++r;
  }
  return r;
}

std::string arch_name(int device) {
  hipDeviceProp_t prop;
  RSB_HIP(hipGetDeviceProperties(&prop, device));
  std::string a(prop.gcnArchName);
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

TileKey make_key(const std::string &arch, int prec, int lr, int nz, int ls, int m, int s) {
  char b[160];
  std::snprintf(b, sizeof(b), "%s %d %d %d %d %d %d", arch.c_str(), prec, lr, nz, ls, m, s);
  return b;
}

bool valid_rpt(int r) {
  for (int c : kCandidates)
    if (c == r) return true;
  return false;
}

void read_cache(const std::string &path) {
  if (g_files_read.count(path)) return;
  g_files_read[path] = true;
  FILE *f = std::fopen(path.c_str(), "r");
  if (!f) return;  // a missing file is an empty cache
  char arch[64];
  int ver, prec, lr, nz, ls, m, st, rpt;
  char line[256];
  while (std::fgets(line, sizeof(line), f)) {
    // (lines of other versions are ignored: version 1 had no step count)
    if (std::sscanf(line, "rsb-tile %d %63s %d %d %d %d %d %d %d", &ver, arch, &prec, &lr, &nz,
                    &ls, &m, &st, &rpt) == 9 &&
        ver == 2 && (st == 1 || st == 2) && valid_rpt(rpt))
      g_tiles[make_key(arch, prec, lr, nz, ls, m, st)] = rpt;
  }
  std::fclose(f);
}

void append_cache(const std::string &path, const TileKey &k, int rpt) {
  FILE *f = std::fopen(path.c_str(), "a");
  if (!f) fail(RSB_EINVAL, "autotune_cache: cannot open " + path + " for appending");
  std::fprintf(f, "rsb-tile 2 %s %d\n", k.c_str(), rpt);
  std::fclose(f);
}

// The launch sequence the solve will run: two steps at a time with
// lanczos_s = 2 (thick restart, sliced ELL), else one.
bool two_step(const rsb_opts &o) {
  return o.lanczos_s == 2 && o.lanczos_keep > 0 && !o.gather_scatter;
}

double trial(Level &L, int rpt, const rsb_opts &o, void *work, Ctx &ctx) {
  level_tables(L, rpt, ctx);
  const LevelView v = view_of(L);
  const bool pairs = two_step(o);
  return o.precision == RSB_MIXED ? lanczos_trial_ms<float>(v, o.lanczos_m, pairs, work, ctx)
                                  : lanczos_trial_ms<double>(v, o.lanczos_m, pairs, work, ctx);
}

}  // namespace

int default_rpt(int64_t) { return 4; }

void choose_tile(Level &L, const rsb_opts &o, void *work, Ctx &ctx) {
  int want;
  if (o.rows_per_thread) {
    want = o.rows_per_thread;
  } else if (o.autotune == 0 || o.method == RSB_INVERSE_CG || o.lanczos_m < 4) {
    want = default_rpt(L.nrows);
  } else {
    const int64_t nnz_row = L.nrows > 0 ? (L.nnz + L.nrows / 2) / L.nrows : 0;
    const TileKey key = make_key(arch_name(ctx.device), o.precision,
                                 ilog2(std::max<int64_t>(L.nrows, 1)), (int)nnz_row,
                                 ilog2(std::max(L.nseg, 1)), o.lanczos_m, two_step(o) ? 2 : 1);
    const std::string path = o.autotune_cache ? o.autotune_cache : "";
    std::lock_guard<std::mutex> lock(g_tune_mu);
    if (!path.empty()) read_cache(path);
    auto it = g_tiles.find(key);
    // autotune 2 times each class once per call, then reuses that choice
    const bool timed_in_call =
        std::find(ctx.tuned.begin(), ctx.tuned.end(), key) != ctx.tuned.end();
    if (it != g_tiles.end() && (o.autotune == 1 || timed_in_call)) {
      want = it->second;
    } else {
      double best = 0.0;
      want = default_rpt(L.nrows);
      for (int c : kCandidates) {
        const double ms = trial(L, c, o, work, ctx);
        if (ctx.verbose >= 2)
          fprintf(stderr, "[rsb]   tile %d rows: %.3f ms per step (two-step form: per pair)\n",
                  kBlock * c, ms);
        if (ms > 0.0 && (best == 0.0 || ms < best)) {
          best = ms;
          want = c;
        }
      }
      g_tiles[key] = want;
      ctx.tuned.push_back(key);
      if (!path.empty()) append_cache(path, key, want);
    }
  }
  if (L.rpt != want || L.blk.empty()) level_tables(L, want, ctx);
}

}  // namespace rsb
