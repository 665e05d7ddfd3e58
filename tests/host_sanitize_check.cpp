// Host-sanitizer run of the library's host code (built by
// tests/test_sanitizers_cpu.py from every csrc/*.hip file compiled for the
// host only, under AddressSanitizer + UndefinedBehaviorSanitizer or under
// ThreadSanitizer).  No GPU and no device code: argument validation,
// workspace planning over a host buffer (never dereferenced), the tuning
// cache and its file format, and the serving scheduler in simulation mode
// with several submitting and polling threads at once.  Exits non-zero on
// the first failed expectation; the sanitizers abort on their own findings.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <thread>
#include <vector>

#include "lqcd.h"

static int failures = 0;
#define EXPECT(c)                                              \
  do {                                                         \
    if (!(c)) {                                                \
      fprintf(stderr, "FAIL %s:%d: %s (last error: %s)\n", __FILE__, __LINE__, #c, lqcd_last_error()); \
      ++failures;                                              \
    }                                                          \
  } while (0)

static lqcd_geom_desc desc(int x, int y, int z, int t, int bc) {
  lqcd_geom_desc d;
  memset(&d, 0, sizeof(d));
  d.L[0] = x;
  d.L[1] = y;
  d.L[2] = z;
  d.L[3] = t;
  d.bc = bc;
  for (int i = 0; i < 4; ++i) d.theta_re[i] = (i == 3 && bc == LQCD_BC_PERIODIC) ? -1.0 : 1.0;
  return d;
}

static void validation(const char* dir) {
  lqcd_geom_t* g = nullptr;
  lqcd_geom_desc bad = desc(4, 4, 4, 7, LQCD_BC_PERIODIC);
  EXPECT(lqcd_geom(&bad, &g) == LQCD_EINVAL && g == nullptr);
  bad = desc(4, 4, 4, 4, 9);
  EXPECT(lqcd_geom(&bad, &g) == LQCD_EINVAL);
  EXPECT(lqcd_geom(nullptr, &g) == LQCD_EINVAL);
  lqcd_geom_desc d = desc(6, 4, 4, 8, LQCD_BC_SF);
  EXPECT(lqcd_geom(&d, &g) == LQCD_OK && g);
  EXPECT(lqcd_geom_volume(g) == 768);
  EXPECT(lqcd_gauge_bytes(g, LQCD_PM_F64) > 0);
  const int pm = LQCD_PM_F64 | LQCD_PM_F32 | LQCD_PM_BF16;
  const size_t nb = lqcd_ws_bytes(g, pm, 3);
  EXPECT(nb > 0 && lqcd_vec_bytes(g, LQCD_F32, 3, 2) > 0);
  std::vector<unsigned char> buf(nb + 256);
  void* base = (void*)(((uintptr_t)buf.data() + 255) & ~(uintptr_t)255);
  lqcd_ws_t* w = nullptr;
  EXPECT(lqcd_ws_create(g, pm, 3, base, nb, &w) == LQCD_OK);
  lqcd_ws_t* w2 = nullptr;
  EXPECT(lqcd_ws_create(g, pm, 3, base, nb - 1, &w2) == LQCD_ENOMEM && w2 == nullptr);
  lqcd_tuning t = {3, 2, 1, LQCD_TUNE_NT_STORE}, back;
  EXPECT(lqcd_ws_set_tuning(w, LQCD_F32, &t) == LQCD_OK);
  EXPECT(lqcd_ws_get_tuning(w, LQCD_F32, &back) == LQCD_OK && back.nr_tile == 3 && back.block_order == 2);
  t.nr_tile = 4;
  EXPECT(lqcd_ws_set_tuning(w, LQCD_F32, &t) == LQCD_EINVAL);
  int32_t pairs[2] = {15, 16};
  void* fake = (void*)(uintptr_t)(1 << 20);
  EXPECT(lqcd_meson(g, fake, 1, pairs, fake, nullptr, w, nullptr) == LQCD_EINVAL);
  EXPECT(strstr(lqcd_last_error(), "gamma mask") != nullptr);
  EXPECT(lqcd_meson_noalloc(g, fake, 40, pairs, fake, nullptr, nullptr) == LQCD_EINVAL);
  lqcd_ws_free(w);
  lqcd_geom_free(g);
  lqcd_geom_desc big = desc(32, 32, 32, 80, LQCD_BC_PERIODIC);
  EXPECT(lqcd_geom(&big, &g) == LQCD_OK);
  pairs[1] = 15;
  EXPECT(lqcd_meson_noalloc(g, fake, 1, pairs, fake, nullptr, nullptr) == LQCD_EINVAL);
  lqcd_geom_free(g);
  EXPECT(lqcd_solve(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == LQCD_EINVAL);
  EXPECT(strcmp(lqcd_strerror(LQCD_ENOCONV), "solver did not converge") == 0);

  // tuning cache file: load, save, reload, malformed, missing
  char path[4096], out[4096];
  snprintf(path, sizeof(path), "%s/tune_in.txt", dir);
  snprintf(out, sizeof(out), "%s/tune_out.txt", dir);
  FILE* f = fopen(path, "w");
  fprintf(f, "# lqcd tuning cache v1\n");
  fprintf(f, "gfx950 32 32 32 64 0 1 2 12 0 0 3 2 1 1 812.500\n");
  fprintf(f, "gfx950 16 16 16 32 0 1 0 1 0 1 1 1 1 19 25.125\n");
  fclose(f);
  lqcd_tune_cache_clear();
  EXPECT(lqcd_tune_cache_load(path) == LQCD_OK && lqcd_tune_cache_size() == 2);
  EXPECT(lqcd_tune_cache_save(out) == LQCD_OK);
  lqcd_tune_cache_clear();
  EXPECT(lqcd_tune_cache_load(out) == LQCD_OK && lqcd_tune_cache_size() == 2);
  f = fopen(path, "w");
  fprintf(f, "gfx950 8 8 8 8 0 1 2 12 0 0 9 2 1 1 1.0\n");
  fclose(f);
  EXPECT(lqcd_tune_cache_load(path) == LQCD_EINVAL && lqcd_tune_cache_size() == 2);
  snprintf(path, sizeof(path), "%s/missing.txt", dir);
  EXPECT(lqcd_tune_cache_load(path) == LQCD_ENOTFOUND);
  lqcd_tune_cache_clear();
}

// serving scheduler, simulation mode: submitters, pollers, stop, destroy
static void serving() {
  lqcd_server_t* s = nullptr;
  EXPECT(lqcd_server_create(nullptr, (size_t)1 << 40, 4, 64, 0.002, &s) == LQCD_OK);
  int g8 = -1, g16 = -1;
  lqcd_geom_desc d8 = desc(8, 8, 8, 8, LQCD_BC_PERIODIC), d16 = desc(16, 16, 16, 32, LQCD_BC_OPEN);
  EXPECT(lqcd_server_add_gauge(s, &d8, nullptr, LQCD_PM_F64 | LQCD_PM_F32, &g8) == LQCD_OK);
  EXPECT(lqcd_server_add_gauge(s, &d16, nullptr, LQCD_PM_F64 | LQCD_PM_F32, &g16) == LQCD_OK);
  EXPECT(lqcd_server_warmup(s, g8, LQCD_F32, 1) == LQCD_OK);
  // four submitting threads and two polling threads at once; tickets pass
  // from the submitters to the pollers through a mutex-guarded list
  const int kThreads = 4, kPer = 40, kTotal = kThreads * kPer;
  std::mutex mu;
  std::vector<uint64_t> pending;
  std::atomic<int> submitted{0}, done{0}, busy{0};
  std::vector<std::thread> th;
  for (int i = 0; i < kThreads; ++i)
    th.emplace_back([&, i]() {
      for (int k = 0; k < kPer; ++k) {
        lqcd_solve_params p;
        memset(&p, 0, sizeof(p));
        p.d.kappa = 0.125 + 0.001 * k;
        p.d.csw = 1.9;
        p.d.cF = 1.0;
        p.solver = LQCD_SOLVER_CG_EO;
        p.inner_prec = ((k + i) % 2) ? LQCD_F32 : LQCD_F64;
        p.maxiter = 100;
        p.tol = 1e-10;
        p.nrhs = (k % 3 == 0) ? 12 : 1;
        uint64_t tk = 0;
        int rc;
        while ((rc = lqcd_submit(s, (k % 4) ? g8 : g16, &p, nullptr, nullptr, &tk)) == LQCD_EBUSY) {
          busy++;
          std::this_thread::yield();
        }
        EXPECT(rc == LQCD_OK);
        submitted++;
        if (rc != LQCD_OK) {  // nothing to poll: count it as finished
          done++;
          continue;
        }
        std::lock_guard<std::mutex> lk(mu);
        pending.push_back(tk);
      }
    });
  for (int h = 0; h < 2; ++h)
    th.emplace_back([&]() {
      std::vector<lqcd_solve_info> info(12);
      double times[3];
      while (done.load() < kTotal) {
        uint64_t tk = 0;
        {
          std::lock_guard<std::mutex> lk(mu);
          if (!pending.empty()) {
            tk = pending.back();
            pending.pop_back();
          }
        }
        if (!tk) {
          std::this_thread::yield();
          continue;
        }
        const int rc = lqcd_poll(s, tk, info.data(), times);
        if (rc == LQCD_PENDING) {
          std::lock_guard<std::mutex> lk(mu);
          pending.insert(pending.begin(), tk);
          continue;
        }
        EXPECT(rc == LQCD_OK);
        EXPECT(times[0] <= times[1] && times[1] <= times[2]);
        done++;
      }
    });
  for (auto& t : th) t.join();
  EXPECT(done.load() == kTotal && submitted.load() == kTotal);
  // a queue left behind is cancelled by destroy
  lqcd_solve_params p;
  memset(&p, 0, sizeof(p));
  p.d.kappa = 0.13;
  p.d.csw = 1.9;
  p.d.cF = 1.0;
  p.solver = LQCD_SOLVER_CG_EO;
  p.maxiter = 10;
  p.tol = 1e-10;
  p.nrhs = 1;
  uint64_t tk;
  for (int k = 0; k < 20; ++k) (void)lqcd_submit(s, g8, &p, nullptr, nullptr, &tk);
  EXPECT(lqcd_server_destroy(s, 1) == LQCD_OK);
  printf("serving: %d requests, %d busy retries\n", kThreads * kPer, busy.load());
}

int main(int argc, char** argv) {
  const char* dir = argc > 1 ? argv[1] : "/tmp";
  validation(dir);
  serving();
  printf("%s\n", failures ? "FAILED" : "all ok");
  return failures ? 1 : 0;
}
