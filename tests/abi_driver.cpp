// Host-side checks of every C entry point, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code: argument validation, error
// codes, workspace sizes and the exchange-grid rule.  No device is needed:
// each call either fails validation or stops at the device query.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fock.h"
#include "../paper_1305_7313_amd/csrc/tune_cache.h"

static int fails = 0;
#define EXPECT(cond)                                            \
  do {                                                          \
    if (!(cond)) {                                              \
      std::printf("FAIL line %d: %s\n", __LINE__, #cond);      \
      ++fails;                                                  \
    }                                                           \
  } while (0)

static bool reached_device_or_ok(fock_status st) { return st == FOCK_OK || st == FOCK_E_HIP; }

int main(int argc, char** argv) {
  // cubic 10 bohr cell, 24^3 grid, sphere |m|^2 <= 25 (alias-free: |m_a| <= 5)
  std::vector<int32_t> mill;
  for (int a = -5; a <= 5; ++a)
    for (int b = -5; b <= 5; ++b)
      for (int c = -5; c <= 5; ++c)
        if (a * a + b * b + c * c <= 25) {
          mill.push_back(a);
          mill.push_back(b);
          mill.push_back(c);
        }
  fock_cell cell{};
  for (int k = 0; k < 3; ++k) {
    cell.a[k][k] = 10.0;
    cell.n[k] = 24;
    cell.nq[k] = 1;
  }
  cell.npw = (int32_t)(mill.size() / 3);
  cell.miller = mill.data();
  fock_orbs o{};
  o.c = reinterpret_cast<const void*>(0x1000);
  o.w = reinterpret_cast<const double*>(0x2000);
  o.nb = 4;
  o.ld = cell.npw;
  const double q0[3] = {0.0, 0.0, 0.0};
  void* ws = reinterpret_cast<void*>(0x4000);
  void* out = reinterpret_cast<void*>(0x3000);
  double* ex = reinterpret_cast<double*>(0x5000);
  const size_t big = (size_t)1 << 40;

  // workspace sizes
  EXPECT(fock_workspace_size(&cell, FOCK_C128, 4, 4) > 0);
  EXPECT(fock_workspace_size(&cell, FOCK_C64, 4, 4) < fock_workspace_size(&cell, FOCK_C128, 4, 4));
  EXPECT(fock_workspace_size(&cell, 9, 4, 4) == 0);
  EXPECT(fock_workspace_size(nullptr, FOCK_C128, 4, 4) == 0);
  EXPECT(fock_workspace_size_kmesh(&cell, FOCK_C64, 8, 4) > 0);
  EXPECT(fock_workspace_size_gamma(&cell, FOCK_C128, 5) > 0);
  EXPECT(fock_band_workspace_size(&cell, FOCK_C128, 70) > 0);

  // fock_apply: argument errors in validation order, then the device query
  EXPECT(fock_apply(nullptr, q0, FOCK_C128, &o, &o, out, ws, big, nullptr) == FOCK_E_ARG);
  EXPECT(fock_apply(&cell, q0, 7, &o, &o, out, ws, big, nullptr) == FOCK_E_ARG);
  fock_orbs bad = o;
  bad.ld = cell.npw - 1;
  EXPECT(fock_apply(&cell, q0, FOCK_C128, &bad, &o, out, ws, big, nullptr) == FOCK_E_ARG);
  bad = o;
  bad.nb = -1;
  EXPECT(fock_apply(&cell, q0, FOCK_C128, &o, &bad, out, ws, big, nullptr) == FOCK_E_ARG);
  const double qlat[3] = {2.0 * 3.14159265358979323846 / 10.0, 0.0, 0.0};
  EXPECT(fock_apply(&cell, qlat, FOCK_C128, &o, &o, out, ws, big, nullptr) == FOCK_E_SINGULAR_Q);
  EXPECT(fock_apply(&cell, q0, FOCK_C128, &o, &o, out, ws, 16, nullptr) == FOCK_E_WORKSPACE);
  EXPECT(std::strlen(fock_last_error()) > 0);
  EXPECT(reached_device_or_ok(fock_apply(&cell, q0, FOCK_C128, &o, &o, out, ws, big, nullptr)));
  fock_cell odd = cell;
  odd.n[0] = 20;
  EXPECT(fock_apply(&odd, q0, FOCK_C128, &o, &o, out, ws, big, nullptr) == FOCK_E_UNSUPPORTED_GRID);
  // a sphere too large for the grid without a cutoff aliases; with E_fock = E_wfc it does not
  std::vector<int32_t> wide = mill;
  wide[0] = 6;
  fock_cell wc = cell;
  wc.miller = wide.data();
  EXPECT(fock_apply(&wc, q0, FOCK_C128, &o, &o, out, ws, big, nullptr) == FOCK_E_ALIAS);
  fock_cell red = cell;
  red.ecut_fock = 25.0 * (2.0 * 3.14159265358979323846 / 10.0) * (2.0 * 3.14159265358979323846 / 10.0);
  EXPECT(reached_device_or_ok(fock_apply(&red, q0, FOCK_C128, &o, &o, out, ws, big, nullptr)));

  // allocation-free apply: same validation; requests beyond the fixed scratch array are refused on the host
  EXPECT(fock_apply_noalloc(nullptr, q0, FOCK_C128, &o, &o, out, nullptr) == FOCK_E_ARG);
  EXPECT(fock_apply_noalloc(&cell, q0, 5, &o, &o, out, nullptr) == FOCK_E_ARG);
  EXPECT(fock_apply_noalloc(&cell, qlat, FOCK_C128, &o, &o, out, nullptr) == FOCK_E_SINGULAR_Q);
  EXPECT(fock_apply_noalloc(&cell, q0, FOCK_C128, &o, &o, nullptr, nullptr) == FOCK_E_ARG);
  EXPECT(fock_apply_noalloc(&wc, q0, FOCK_C128, &o, &o, out, nullptr) == FOCK_E_ALIAS);
  {
    fock_orbs many = o;
    many.nb = 64;  // a 16 x 16 pair tile of 24^3 FP64 boxes alone is 56 MB
    EXPECT(fock_apply_noalloc(&cell, q0, FOCK_C128, &many, &many, out, nullptr) == FOCK_E_WORKSPACE);
    EXPECT(std::strstr(fock_last_error(), "scratch") != nullptr);
  }
  EXPECT(reached_device_or_ok(fock_apply_noalloc(&cell, q0, FOCK_C128, &o, &o, out, nullptr)));

  // energies, gradients, k-mesh, Gamma, band loops
  EXPECT(fock_energy(&cell, q0, FOCK_C64, &o, &o, nullptr, ws, big, nullptr) != FOCK_OK);
  EXPECT(reached_device_or_ok(fock_energy(&cell, q0, FOCK_C64, &o, &o, ex, ws, big, nullptr)));
  EXPECT(reached_device_or_ok(
      fock_energy_backward(&cell, q0, FOCK_C128, &o, &o, ex, out, out, ws, big, nullptr)));
  const double kpts[6] = {0.0, 0.0, 0.0, 0.31, 0.0, 0.0};
  fock_orbs sets[2] = {o, o};
  EXPECT(fock_energy_kmesh(&cell, 0, kpts, FOCK_C64, sets, ex, ws, big, nullptr) == FOCK_E_ARG);
  EXPECT(reached_device_or_ok(fock_energy_kmesh(&cell, 2, kpts, FOCK_C64, sets, ex, ws, big, nullptr)));
  void* grads[2] = {out, out};
  EXPECT(reached_device_or_ok(
      fock_energy_kmesh_backward(&cell, 2, kpts, FOCK_C64, sets, ex, grads, ws, big, nullptr)));
  EXPECT(fock_energy_kmesh_grad(&cell, 2, kpts, FOCK_C64, sets, nullptr, grads, ws, big, nullptr) == FOCK_E_ARG);
  void* half[2] = {out, nullptr};
  EXPECT(fock_energy_kmesh_grad(&cell, 2, kpts, FOCK_C64, sets, ex, half, ws, big, nullptr) == FOCK_E_ARG);
  EXPECT(fock_energy_kmesh_grad(&cell, 2, kpts, FOCK_C64, sets, ex, grads, ws, 64, nullptr) == FOCK_E_WORKSPACE);
  EXPECT(reached_device_or_ok(fock_energy_kmesh_grad(&cell, 2, kpts, FOCK_C64, sets, ex, grads, ws, big, nullptr)));
  EXPECT(fock_apply_gamma(&cell, FOCK_C128, &o, out, ws, 8, nullptr) == FOCK_E_WORKSPACE);
  EXPECT(reached_device_or_ok(fock_apply_gamma(&cell, FOCK_C128, &o, out, ws, big, nullptr)));
  EXPECT(fock_band_density(&cell, FOCK_C128, &o, nullptr, ws, big, nullptr) != FOCK_OK);
  EXPECT(reached_device_or_ok(fock_band_density(&cell, FOCK_C128, &o, ex, ws, big, nullptr)));
  EXPECT(fock_band_force(&cell, nullptr, FOCK_C128, &o, ws, out, ws, big, nullptr) == FOCK_E_ARG);
  EXPECT(reached_device_or_ok(fock_band_force(&cell, q0, FOCK_C64, &o, ws, out, ws, big, nullptr)));

  // exchange grid rule
  int32_t n[3] = {0, 0, 0};
  EXPECT(fock_exchange_grid(&red, 0, nullptr, FOCK_C128, n) == FOCK_OK);
  EXPECT(n[0] == 24 && n[1] == 24 && n[2] == 24);
  EXPECT(fock_exchange_grid(&red, 1, nullptr, FOCK_C128, n) == FOCK_E_ARG);
  EXPECT(fock_exchange_grid(nullptr, 0, nullptr, FOCK_C128, n) == FOCK_E_ARG);

  // batched form
  void* plan = nullptr;
  EXPECT(fock_batch_plan_create(nullptr, &o, nullptr, nullptr, 1, FOCK_C128, nullptr, &plan) == FOCK_E_ARG);
  EXPECT(fock_batch_plan_create(&cell, &o, nullptr, nullptr, 0, FOCK_C128, nullptr, &plan) == FOCK_E_ARG);
  EXPECT(fock_batch_plan_create(&cell, &o, nullptr, nullptr, 1, 3, nullptr, &plan) == FOCK_E_ARG);
  EXPECT(fock_batch_plan_create(&cell, &o, nullptr, &qlat, 1, FOCK_C128, nullptr, &plan) == FOCK_E_SINGULAR_Q);
  EXPECT(plan == nullptr);
  EXPECT(fock_batch_apply(nullptr, nullptr, nullptr, nullptr) == FOCK_E_ARG);

  EXPECT(fock_batch_set_wait_limit(nullptr, 1.0) == FOCK_E_ARG);

  // tune cache: entries outside the schedule's ranges are ignored (the batch is tuned again)
  {
    const std::string cache = std::string(argc > 1 ? argv[1] : ".") + "/abi_driver_tune_cache.json";
    const char* path = cache.c_str();
    if (FILE* f = std::fopen(path, "w")) {
      std::fprintf(f,
                   "{\n"
                   "\"ok\": {\"tile\": 8, \"slots\": 6, \"units_per_ticket\": 32, \"blocks_per_cu\": 2, \"ms\": 1.5, \"mode\": 0},\n"
                   "\"old\": {\"tile\": 16, \"slots\": 4, \"units_per_ticket\": 128, \"blocks_per_cu\": 1, \"ms\": 2.0}\n"
                   "\"slots9\": {\"tile\": 16, \"slots\": 9, \"units_per_ticket\": 32, \"blocks_per_cu\": 1, \"ms\": 1, \"mode\": 0},\n"
                   "\"slots0\": {\"tile\": 16, \"slots\": 0, \"units_per_ticket\": 32, \"blocks_per_cu\": 1, \"ms\": 1, \"mode\": 0},\n"
                   "\"slots3\": {\"tile\": 16, \"slots\": 3, \"units_per_ticket\": 32, \"blocks_per_cu\": 1, \"ms\": 1, \"mode\": 0},\n"
                   "\"tile32\": {\"tile\": 32, \"slots\": 6, \"units_per_ticket\": 32, \"blocks_per_cu\": 1, \"ms\": 1, \"mode\": 0},\n"
                   "\"ticket0\": {\"tile\": 16, \"slots\": 6, \"units_per_ticket\": 0, \"blocks_per_cu\": 1, \"ms\": 1, \"mode\": 1},\n"
                   "\"ticketneg\": {\"tile\": 16, \"slots\": 6, \"units_per_ticket\": -4, \"blocks_per_cu\": 1, \"ms\": 1, \"mode\": 1},\n"
                   "\"mode7\": {\"tile\": 16, \"slots\": 6, \"units_per_ticket\": 32, \"blocks_per_cu\": 1, \"ms\": 1, \"mode\": 7},\n"
                   "\"bpc0\": {\"tile\": 16, \"slots\": 6, \"units_per_ticket\": 32, \"blocks_per_cu\": 0, \"ms\": 1, \"mode\": 0},\n"
                   "\"nanms\": {\"tile\": 16, \"slots\": 6, \"units_per_ticket\": 32, \"blocks_per_cu\": 1, \"ms\": nan, \"mode\": 0},\n"
                   "\"branches9\": {\"tile\": 16, \"slots\": 6, \"units_per_ticket\": 32, \"blocks_per_cu\": 1, \"ms\": 1, \"mode\": 1, \"branches\": 9},\n"
                   "\"branches0\": {\"tile\": 16, \"slots\": 6, \"units_per_ticket\": 32, \"blocks_per_cu\": 1, \"ms\": 1, \"mode\": 1, \"branches\": 0},\n"
                   "\"branches3\": {\"tile\": 16, \"slots\": 6, \"units_per_ticket\": 32, \"blocks_per_cu\": 1, \"ms\": 1, \"mode\": 1, \"branches\": 3},\n"
                   "\"short\": {\"tile\": 16, \"slots\": 6},\n"
                   "\"junk\": {garbage},\n"
                   "\"twice\": {\"tile\": 8, \"slots\": 6, \"units_per_ticket\": 32, \"blocks_per_cu\": 1, \"ms\": 1, \"mode\": 0},\n"
                   "\"twice\": {\"tile\": 99, \"slots\": 6, \"units_per_ticket\": 32, \"blocks_per_cu\": 1, \"ms\": 1, \"mode\": 0}\n"
                   "}\n");
      std::fclose(f);
    }
    fockx::BatchParams p;
    EXPECT(fockx::tune_cache_lookup(path, "ok", &p) && p.tile == 8 && p.units_per_ticket == 32 &&
           p.blocks_per_cu == 2 && p.mode == 0);
    EXPECT(fockx::tune_cache_lookup(path, "old", &p) && p.slots == 4 && p.mode == 0);
    EXPECT(fockx::tune_cache_lookup(path, "branches3", &p) && p.mode == 1 && p.branches == 3);
    EXPECT(fockx::tune_cache_lookup(path, "ok", &p) && p.branches == 1);
    for (const char* bad : {"slots9", "slots0", "slots3", "tile32", "ticket0", "ticketneg", "mode7", "bpc0", "nanms",
                            "branches9", "branches0",
                            "short", "junk", "twice", "absent"}) {
      fockx::BatchParams q;
      const bool got = fockx::tune_cache_lookup(path, bad, &q);
      if (got) std::printf("accepted malformed cache entry %s\n", bad);
      EXPECT(!got);
    }
    EXPECT(!fockx::tune_cache_lookup("", "ok", &p));
    EXPECT(!fockx::tune_cache_lookup("no/such/dir/cache.json", "ok", &p));
    // a stored entry reads back; an out-of-range one is never written
    fockx::BatchParams w;
    w.tile = 16;
    w.units_per_ticket = 512;
    w.mode = 1;
    w.branches = 2;
    w.ms = 12.5;
    fockx::tune_cache_store(path, "new", w);
    EXPECT(fockx::tune_cache_lookup(path, "new", &p) && p.units_per_ticket == 512 && p.mode == 1 && p.branches == 2);
    EXPECT(fockx::tune_cache_lookup(path, "ok", &p) && p.tile == 8);
    w.slots = 40;
    fockx::tune_cache_store(path, "bad_store", w);
    EXPECT(!fockx::tune_cache_lookup(path, "bad_store", &p));
    std::remove(path);
  }

  // transforms and strings
  const int32_t grid[3] = {24, 24, 24};
  EXPECT(fock_fft3d(grid, FOCK_C128, 2, out, 1, nullptr) == FOCK_E_ARG);
  const fock_status all[] = {FOCK_OK, FOCK_E_ARG, FOCK_E_ALIAS, FOCK_E_SINGULAR_Q,
                             FOCK_E_WORKSPACE, FOCK_E_UNSUPPORTED_GRID, FOCK_E_HIP};
  for (fock_status st : all) EXPECT(std::strlen(fock_status_string(st)) > 0);
  EXPECT(fock_trace_enable(0) > 0);

  std::printf("abi driver: %d failure(s)\n", fails);
  return fails ? 1 : 0;
}
