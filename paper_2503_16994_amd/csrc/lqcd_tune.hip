// Process-wide cache of hop-kernel tunings.
//
// The autotuner times candidate launch shapes at a lattice's real shape; the
// best one depends on the GPU, the lattice extents and boundary type, the
// storage precision, the rhs count, the link storage (two rows or full), the
// twisted-mass variant and the caller's direction-split choice, and on
// nothing else (no tuning changes a result).  Entries are keyed by exactly
// those; lqcd_autotune adds its result, and a caller that must not tune at
// run time (a serving loop) reads entries filled beforehand, possibly from a
// file written by an earlier process.  All access is under one mutex.
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "lqcd_internal.h"

using namespace lqcd;

namespace {

struct Key {
  std::string arch;
  int L[4];
  int bc, two_row, prec, nrhs, twisted, split;
  auto tie() const { return std::tie(arch, L[0], L[1], L[2], L[3], bc, two_row, prec, nrhs, twisted, split); }
  bool operator<(const Key& o) const { return tie() < o.tie(); }
};

struct Entry {
  lqcd_tuning t;
  double us;
};

std::mutex g_mu;
std::map<Key, Entry> g_cache;

// architecture name of the current device ("gfx950" etc., without feature
// suffixes); empty on failure
std::string device_arch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "";
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

Key make_key(const std::string& arch, const lqcd_geom_desc& d, int two_row, int prec, int nrhs, int twisted,
             int split) {
  Key k;
  k.arch = arch;
  for (int i = 0; i < 4; ++i) k.L[i] = d.L[i];
  k.bc = d.bc;
  k.two_row = two_row ? 1 : 0;
  k.prec = prec;
  k.nrhs = nrhs;
  k.twisted = twisted ? 1 : 0;
  k.split = split ? 1 : 0;
  return k;
}

bool valid_tuning(const lqcd_tuning& t) {
  return t.nr_tile >= 1 && t.nr_tile <= 3 && t.block_order >= 0 && t.block_order <= 6 &&
         (t.rhs_lanes == 1 || t.rhs_lanes == 2 || t.rhs_lanes == 4) &&
         !(t.flags & ~(LQCD_TUNE_NT_STORE | LQCD_TUNE_CACHED_GAUGE | (3 << LQCD_TUNE_OCC_SHIFT) |
                       LQCD_TUNE_DIR_SPLIT));
}

}  // namespace

namespace lqcd {

void tune_cache_put(const lqcd_gauge_t* u, int prec, int nrhs, int twisted, const lqcd_tuning& t, double us) {
  const Key k = make_key(device_arch(), u->g->desc, u->two_row, prec, nrhs, twisted,
                         (t.flags & LQCD_TUNE_DIR_SPLIT) != 0);
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache[k] = Entry{t, us};
}

}  // namespace lqcd

extern "C" int lqcd_tune_cache_find(const lqcd_gauge_t* u, int prec, int nrhs, int twisted, int dir_split,
                                    lqcd_tuning* t) {
  if (!u || !t) return fail(LQCD_EINVAL, "lqcd_tune_cache_find: null pointer");
  if (prec < 0 || prec > 2 || nrhs < 1) return fail(LQCD_EINVAL, "lqcd_tune_cache_find: bad precision or nrhs");
  const Key k = make_key(device_arch(), u->g->desc, u->two_row, prec, nrhs, twisted, dir_split);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_cache.find(k);
  if (it == g_cache.end()) return fail(LQCD_ENOTFOUND, "lqcd_tune_cache_find: no entry");
  *t = it->second.t;
  return LQCD_OK;
}

extern "C" int lqcd_tune_cache_put(const lqcd_gauge_t* u, int prec, int nrhs, int twisted, const lqcd_tuning* t) {
  if (!u || !t) return fail(LQCD_EINVAL, "lqcd_tune_cache_put: null pointer");
  if (prec < 0 || prec > 2 || nrhs < 1 || !valid_tuning(*t))
    return fail(LQCD_EINVAL, "lqcd_tune_cache_put: value out of range");
  tune_cache_put(u, prec, nrhs, twisted, *t, 0.0);
  return LQCD_OK;
}

extern "C" int lqcd_tune_cache_size(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  return (int)g_cache.size();
}

extern "C" void lqcd_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache.clear();
}

// One line per entry:
//   arch L0 L1 L2 L3 bc two_row prec nrhs twisted split nr_tile block_order rhs_lanes flags us
extern "C" int lqcd_tune_cache_save(const char* path) {
  if (!path) return fail(LQCD_EINVAL, "lqcd_tune_cache_save: null path");
  FILE* f = fopen(path, "w");
  if (!f) return fail(LQCD_EINVAL, "lqcd_tune_cache_save: cannot open %s", path);
  std::lock_guard<std::mutex> lk(g_mu);
  fprintf(f, "# lqcd tuning cache v1\n");
  for (const auto& kv : g_cache) {
    const Key& k = kv.first;
    const lqcd_tuning& t = kv.second.t;
    fprintf(f, "%s %d %d %d %d %d %d %d %d %d %d %d %d %d %d %.3f\n", k.arch.c_str(), k.L[0], k.L[1], k.L[2],
            k.L[3], k.bc, k.two_row, k.prec, k.nrhs, k.twisted, k.split, t.nr_tile, t.block_order, t.rhs_lanes,
            t.flags, kv.second.us);
  }
  const bool ok = (fclose(f) == 0);
  return ok ? LQCD_OK : fail(LQCD_EINVAL, "lqcd_tune_cache_save: write error on %s", path);
}

// Adds the entries of a file written by lqcd_tune_cache_save (replacing
// entries with the same key); a malformed line makes the call fail with
// EINVAL and add nothing.
extern "C" int lqcd_tune_cache_load(const char* path) {
  if (!path) return fail(LQCD_EINVAL, "lqcd_tune_cache_load: null path");
  FILE* f = fopen(path, "r");
  if (!f) return fail(LQCD_ENOTFOUND, "lqcd_tune_cache_load: cannot open %s", path);
  std::map<Key, Entry> add;
  char line[512];
  int lineno = 0, rc = LQCD_OK;
  while (fgets(line, sizeof(line), f)) {
    ++lineno;
    if (line[0] == '#' || line[0] == '\n') continue;
    char arch[64];
    Key k;
    lqcd_tuning t;
    double us = 0.0;
    const int n = sscanf(line, "%63s %d %d %d %d %d %d %d %d %d %d %d %d %d %d %lf", arch, &k.L[0], &k.L[1], &k.L[2],
                         &k.L[3], &k.bc, &k.two_row, &k.prec, &k.nrhs, &k.twisted, &k.split, &t.nr_tile,
                         &t.block_order, &t.rhs_lanes, &t.flags, &us);
    if (n != 16 || k.prec < 0 || k.prec > 2 || k.nrhs < 1 || !valid_tuning(t) ||
        ((t.flags & LQCD_TUNE_DIR_SPLIT) != 0) != (k.split != 0)) {
      rc = fail(LQCD_EINVAL, "lqcd_tune_cache_load: %s line %d malformed", path, lineno);
      break;
    }
    k.arch = arch;
    add[k] = Entry{t, us};
  }
  fclose(f);
  if (rc != LQCD_OK) return rc;
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : add) g_cache[kv.first] = kv.second;
  return LQCD_OK;
}
