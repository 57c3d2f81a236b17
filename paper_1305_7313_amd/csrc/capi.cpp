// C ABI of the exact-exchange path: validation, plan cache and the band-pair
// schedule (section 4 and the band-group loop split of section 5).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fock.h"
#include "fock_launch.h"
#include "tune_cache.h"

using namespace fockx;

namespace {

thread_local std::string g_last_error;

fock_status fail(fock_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

// ---------------------------------------------------------------------------
// Per-kernel-class timing with HIP events (off unless fock_trace_enable(1)).
// ---------------------------------------------------------------------------
enum KClass : int {
  KC_A1_SCATTER = 0, KC_A1_PENCIL, KC_A1_PLANE, KC_P1, KC_P2, KC_P2E, KC_P3, KC_P3B,
  KC_A7_PLANE, KC_A7_PENCIL, KC_A7_GATHER, KC_REDUCE, KC_ZERO, KC_BAND_DENS, KC_BAND_VMUL, KC_BAND_GATHER, KC_COUNT
};
const char* const kClassNames[KC_COUNT] = {
    "a1_scatter", "a1_pencil_inv", "a1_plane_inv", "p1_pair_plane_fwd", "p2_pencil_kernel",
    "p2_pencil_energy", "p3_plane_inv_mac", "p3_second", "a7_plane_fwd", "a7_pencil_fwd", "a7_gather",
    "reduce", "zero_fill", "band_plane_density", "band_plane_vmul", "band_force_gather"};

struct Tracer {
  std::mutex m;
  bool on = false;
  struct Rec { int k; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  double ms[KC_COUNT] = {};
  long long n[KC_COUNT] = {};
  hipEvent_t take() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
};
Tracer& tracer() { static Tracer* t = new Tracer(); return *t; }

struct TraceScope {
  int k; hipStream_t s; hipEvent_t a = nullptr, b = nullptr; bool on;
  TraceScope(int kc, hipStream_t st) : k(kc), s(st) {
    Tracer& T = tracer();
    on = T.on;
    if (on) {
      std::lock_guard<std::mutex> lk(T.m);
      a = T.take(); b = T.take();
      (void)hipEventRecord(a, s);
    }
  }
  ~TraceScope() {
    if (!on) return;
    Tracer& T = tracer();
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(T.m);
    T.recs.push_back({k, a, b});
  }
};
#define FX_TRACE(kc) TraceScope trace_scope_##__LINE__(kc, s)
#define FX_TRACE_S(kc) TraceScope trace_scope_s(kc, s)

// ---------------------------------------------------------------------------
// Plans: per device, grid, lattice, dtype and sphere.
// ---------------------------------------------------------------------------
struct Plan {
  int device = 0;
  int n[3] = {0, 0, 0};
  long long N = 0;
  int dtype = 0;
  double a[3][3];
  double b[3][3];
  double omega = 0.0;
  int npw = 0;
  int* d_slot = nullptr;        // [npw] flat box index of each sphere G
  void* d_tw[3] = {nullptr, nullptr, nullptr};  // per axis, length n_a, dtype precision
  // [n3] per plane column i3: pair densities (support S - S) have no component
  // (after the transform over the plane axes) at rows |m2| > d_live[i3]; -1:
  // none in that column.  Null when S - S wraps on this grid.
  signed char* d_live = nullptr;
  bool owns = true;  // false: the device tables live in memory the plan does not own
  ~Plan() {
    if (!owns) return;
    (void)hipSetDevice(device);
    if (d_slot) (void)hipFree(d_slot);
    if (d_live) (void)hipFree(d_live);
    for (auto p : d_tw)
      if (p) (void)hipFree(p);
  }
};

using PlanKey = std::tuple<int, int, int, int, int, int, uint64_t, std::string>;
// Heap-held and never destroyed at exit: device frees after the HIP runtime
// has shut down are not safe.  fock_release_plans() frees them explicitly.
std::mutex g_mutex;
auto& g_plans = *new std::map<PlanKey, std::shared_ptr<Plan>>();
auto& g_fft_plans = *new std::map<std::tuple<int, int, int>, std::shared_ptr<Plan>>();

uint64_t fnv1a(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t k = 0; k < n; ++k) {
    h ^= c[k];
    h *= 1099511628211ull;
  }
  return h;
}

bool size_ok(int n) { return pencil_supported(n); }

void reciprocal(const double a[3][3], double b[3][3], double* omega) {
  const double det = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
                     a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
                     a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
  *omega = std::fabs(det);
  // b_i = 2 pi (a_j x a_k) / det
  const double s = 2.0 * kPi / det;
  for (int i = 0; i < 3; ++i) {
    const double* u = a[(i + 1) % 3];
    const double* v = a[(i + 2) % 3];
    b[i][0] = s * (u[1] * v[2] - u[2] * v[1]);
    b[i][1] = s * (u[2] * v[0] - u[0] * v[2]);
    b[i][2] = s * (u[0] * v[1] - u[1] * v[0]);
  }
}

// tw[m] = exp(-2 pi i m / n), computed in FP64, rounded once for FP32; as
// the bytes of the dtype's complex array.
std::vector<unsigned char> host_twiddles(int n, int dtype) {
  std::vector<unsigned char> out((size_t)n * (dtype == FOCK_C128 ? 16 : 8));
  for (int m = 0; m < n; ++m) {
    const CosSin cs = cossin_2pi(m, n);
    if (dtype == FOCK_C128) {
      const double v[2] = {cs.c, -cs.s};
      std::memcpy(out.data() + 16 * (size_t)m, v, sizeof v);
    } else {
      const float v[2] = {(float)cs.c, (float)(-cs.s)};
      std::memcpy(out.data() + 8 * (size_t)m, v, sizeof v);
    }
  }
  return out;
}

hipError_t upload_twiddles(int n, int dtype, void** out) {
  const std::vector<unsigned char> t = host_twiddles(n, dtype);
  hipError_t e = hipMalloc(out, t.size());
  if (e != hipSuccess) return e;
  return hipMemcpy(*out, t.data(), t.size(), hipMemcpyHostToDevice);
}

int tbytes_of(int dtype) { return dtype == FOCK_C128 ? 8 : 4; }

bool grid_supported(const int n[3], int dtype) {
  if (!size_ok(n[0]) || !plane_supported(n[1], n[2])) return false;
  const int cb = pencil_columns(n[0], tbytes_of(dtype));
  return cb > 0 && (n[1] * n[2]) % cb == 0;
}

std::string grid_str(const int n[3]) {
  char buf[96];
  std::snprintf(buf, sizeof buf, "%dx%dx%d", n[0], n[1], n[2]);
  return buf;
}

fock_status make_fft_plan(const int n[3], int dtype, std::shared_ptr<Plan>* out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(FOCK_E_HIP, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(g_mutex);
  auto key = std::make_tuple(dev * 4 + dtype, n[0], n[1] * 1000 + n[2]);
  auto it = g_fft_plans.find(key);
  if (it != g_fft_plans.end()) {
    *out = it->second;
    return FOCK_OK;
  }
  auto p = std::make_shared<Plan>();
  p->device = dev;
  for (int k = 0; k < 3; ++k) p->n[k] = n[k];
  p->N = (long long)n[0] * n[1] * n[2];
  p->dtype = dtype;
  for (int k = 0; k < 3; ++k) {
    hipError_t e = upload_twiddles(n[k], dtype, &p->d_tw[k]);
    if (e != hipSuccess) return fail(FOCK_E_HIP, std::string("twiddle upload: ") + hipGetErrorString(e));
  }
  g_fft_plans[key] = p;
  *out = p;
  return FOCK_OK;
}

// Validates the cell and returns (creating if needed) its plan.
// Columns of the plane axes (i2, i3) that a pair density can occupy.  The
// sphere S projects onto the plane as a set whose rows, for each m3, span
// [lo(m3), hi(m3)]; a pair density conj(phi) psi lives on S - S, whose column
// m3a - m3b reaches |m2| <= max(hi(m3a) - lo(m3b), hi(m3b) - lo(m3a)).  Out:
// per grid column i3 that bound (-1: empty column).  False when S - S wraps
// on the grid (2 |m| > n - 1 on a plane axis), where every column is kept.
bool pair_columns(const fock_cell* cell, std::vector<signed char>* out) {
  const int n2 = cell->n[1], n3 = cell->n[2];
  std::map<int, std::pair<int, int>> rows;  // m3 -> [lo, hi] of m2 in the projection of S
  for (int p = 0; p < cell->npw; ++p) {
    const int m2 = cell->miller[3 * p + 1], m3 = cell->miller[3 * p + 2];
    auto it = rows.find(m3);
    if (it == rows.end()) rows[m3] = {m2, m2};
    else it->second = {std::min(it->second.first, m2), std::max(it->second.second, m2)};
  }
  std::map<int, int> h;  // d3 -> largest |d2|
  for (const auto& a : rows)
    for (const auto& b : rows) {
      const int d3 = a.first - b.first;
      const int d2 = std::max(a.second.second - b.second.first, b.second.second - a.second.first);
      auto it = h.find(d3);
      if (it == h.end() || it->second < d2) h[d3] = d2;
    }
  out->assign((size_t)n3, (signed char)-1);
  for (const auto& e : h) {
    if (2 * std::abs(e.first) > n3 - 1 || 2 * e.second > n2 - 1 || e.second > 127) return false;
    (*out)[(size_t)((e.first % n3 + n3) % n3)] = (signed char)e.second;
  }
  return true;
}

// Host checks of the cell fields a plan depends on; the reciprocal lattice
// and the volume.
fock_status check_plan_cell(const fock_cell* cell, int dtype, double b[3][3], double* omega) {
  if (!cell) return fail(FOCK_E_ARG, "cell is NULL");
  if (dtype != FOCK_C128 && dtype != FOCK_C64) return fail(FOCK_E_ARG, "dtype must be FOCK_C128 or FOCK_C64");
  for (int k = 0; k < 3; ++k)
    if (cell->n[k] <= 0) return fail(FOCK_E_ARG, "grid sizes must be positive");
  if (!grid_supported(cell->n, dtype))
    return fail(FOCK_E_UNSUPPORTED_GRID, "no compiled transforms for grid " + grid_str(cell->n));
  if (cell->npw <= 0 || !cell->miller) return fail(FOCK_E_ARG, "empty G-sphere (npw <= 0 or miller NULL)");
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      if (!std::isfinite(cell->a[i][j])) return fail(FOCK_E_ARG, "lattice vectors must be finite");
  double om = 0.0;
  reciprocal(cell->a, b, &om);
  if (!(om > 1e-12)) return fail(FOCK_E_ARG, "cell volume is not positive");
  if (cell->g0 != FOCK_G0_ZERO && cell->g0 != FOCK_G0_GB) return fail(FOCK_E_ARG, "g0 must be ZERO or GB");
  if (cell->g0 == FOCK_G0_GB) {
    if (!(cell->gb_alpha > 0.0) || !std::isfinite(cell->gb_alpha)) return fail(FOCK_E_ARG, "gb_alpha must be > 0");
    for (int k = 0; k < 3; ++k)
      if (cell->nq[k] < 1) return fail(FOCK_E_ARG, "nq must be >= 1");
  }
  if (std::isnan(cell->ecut_fock)) return fail(FOCK_E_ARG, "ecut_fock is NaN");
  *omega = om;
  return FOCK_OK;
}

// Sphere tables: the box slot of every G (each G its own slot, inside the
// box) and the live plane columns of a pair density (has_live false when
// S - S wraps on the grid).
fock_status sphere_tables(const fock_cell* cell, std::vector<int>* slot, std::vector<signed char>* live,
                          bool* has_live) {
  const long long N = (long long)cell->n[0] * cell->n[1] * cell->n[2];
  slot->assign((size_t)cell->npw, 0);
  std::vector<unsigned char> seen((size_t)N, 0);
  for (int p = 0; p < cell->npw; ++p) {
    int idx[3];
    for (int k = 0; k < 3; ++k) {
      const int m = cell->miller[3 * p + k];
      if (2 * (long long)std::abs(m) > (long long)cell->n[k] - 1) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "Miller index %d on axis %d does not fit the box n=%d", m, k, cell->n[k]);
        return fail(FOCK_E_ALIAS, buf);
      }
      idx[k] = (m % cell->n[k] + cell->n[k]) % cell->n[k];
    }
    const long long flat = ((long long)idx[0] * cell->n[1] + idx[1]) * cell->n[2] + idx[2];
    if (seen[flat]) return fail(FOCK_E_ALIAS, "repeated G-vector in the sphere list");
    seen[flat] = 1;
    (*slot)[p] = (int)flat;
  }
  *has_live = pair_columns(cell, live);
  return FOCK_OK;
}

fock_status get_plan(const fock_cell* cell, int dtype, std::shared_ptr<Plan>* out) {
  double b[3][3], omega = 0.0;
  fock_status st0 = check_plan_cell(cell, dtype, b, &omega);
  if (st0 != FOCK_OK) return st0;
  int dev = 0;
  const bool have_dev = hipGetDevice(&dev) == hipSuccess;
  const size_t mbytes = (size_t)cell->npw * 3 * sizeof(int32_t);
  const uint64_t h = fnv1a(cell->miller, mbytes);
  std::string akey(reinterpret_cast<const char*>(cell->a), sizeof(cell->a));
  PlanKey key(dev, dtype, cell->n[0], cell->n[1], cell->n[2], cell->npw, h, akey);
  if (have_dev) {
    std::lock_guard<std::mutex> lk(g_mutex);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
      *out = it->second;
      return FOCK_OK;
    }
  }
  // Sphere check (host only): every G has its own box slot.  Whether pair
  // products alias depends on q and the cutoff: check_alias, per call.
  const long long N = (long long)cell->n[0] * cell->n[1] * cell->n[2];
  std::vector<int> slot;
  std::vector<signed char> live;
  bool has_live = false;
  if ((st0 = sphere_tables(cell, &slot, &live, &has_live)) != FOCK_OK) return st0;
  if (!have_dev) return fail(FOCK_E_HIP, "no HIP device available");
  auto p = std::make_shared<Plan>();
  p->device = dev;
  for (int k = 0; k < 3; ++k) p->n[k] = cell->n[k];
  p->N = N;
  p->dtype = dtype;
  std::memcpy(p->a, cell->a, sizeof(p->a));
  std::memcpy(p->b, b, sizeof(b));
  p->omega = omega;
  p->npw = cell->npw;
  hipError_t e = hipMalloc(&p->d_slot, sizeof(int) * (size_t)cell->npw);
  if (e == hipSuccess) e = hipMemcpy(p->d_slot, slot.data(), sizeof(int) * (size_t)cell->npw, hipMemcpyHostToDevice);
  if (e == hipSuccess && has_live) {
    e = hipMalloc(&p->d_live, live.size());
    if (e == hipSuccess) e = hipMemcpy(p->d_live, live.data(), live.size(), hipMemcpyHostToDevice);
  }
  for (int k = 0; k < 3 && e == hipSuccess; ++k) e = upload_twiddles(cell->n[k], dtype, &p->d_tw[k]);
  if (e != hipSuccess) return fail(FOCK_E_HIP, std::string("plan upload: ") + hipGetErrorString(e));
  std::lock_guard<std::mutex> lk(g_mutex);
  g_plans[key] = p;
  *out = p;
  return FOCK_OK;
}

// ---------------------------------------------------------------------------
// Tiling and workspace layout
// ---------------------------------------------------------------------------
constexpr int kGbParts = 512;

struct Tiles {
  int ti, tj;
};
// Pair tile of a job: the block split into the fewest tiles of at most
// pair_tile(element size) orbitals, of near-equal size (174 orbitals at edge
// 32: tiles of 29, not five of 32 and one of 14), so that no launch carries
// a thin remainder.
int balanced_edge(int n, int edge) {
  if (n <= 0) return 1;
  const int parts = (n + edge - 1) / edge;
  return (n + parts - 1) / parts;
}
Tiles tiles_for(int n_occ, int n_tgt, int cplx_bytes) {
  const int edge = pair_tile(cplx_bytes);
  Tiles t;
  t.ti = balanced_edge(n_occ, edge);
  t.tj = balanced_edge(n_tgt, edge);
  return t;
}
// Workspace bounds for any job on blocks of up to nmax orbitals: no tile edge
// exceeds min(nmax, edge) (the balanced edge is not monotonic in n), and a
// block of n orbitals has ceil(n / edge) tiles along it.
int tile_cap(int nmax, int cplx_bytes) { return std::max(1, std::min(nmax, pair_tile(cplx_bytes))); }
int tile_count(int n, int cplx_bytes) { return n > 0 ? (n + pair_tile(cplx_bytes) - 1) / pair_tile(cplx_bytes) : 1; }

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t phiA, phiB, acc, w, epart, tile_e, k0, gbpart, total;
};

Layout layout(long long N, int cplx_bytes, int ngroups, int n_occ, int n_tgt) {
  // Sized for both role orders (the backward pass swaps the blocks).
  const int nmax = n_occ > n_tgt ? n_occ : n_tgt;
  const int tc = tile_cap(nmax, cplx_bytes);
  const size_t nb = (size_t)N * cplx_bytes;
  const int ntiles = tile_count(n_occ, cplx_bytes) * tile_count(n_tgt, cplx_bytes);
  Layout L;
  size_t off = 0;
  L.phiA = off; off += align_up(nb * (size_t)nmax);
  L.phiB = off; off += align_up(nb * (size_t)nmax);
  L.acc = off; off += align_up(nb * (size_t)tc);
  L.w = off; off += align_up(nb * (size_t)tc * tc);
  L.epart = off; off += align_up(sizeof(double) * (size_t)tc * tc * ngroups);
  L.tile_e = off; off += align_up(sizeof(double) * (size_t)ntiles);
  L.k0 = off; off += align_up(sizeof(double));
  L.gbpart = off; off += align_up(sizeof(double) * kGbParts);
  L.total = off;
  return L;
}

// Gamma apply: packed orbitals and packed accumulators ([ceil(nb/2)][N] each)
// and a pair buffer for one packed tile (up to 16 real x 8 packed).
Layout layout_gamma(long long N, int cplx_bytes, int nb) {
  const int m = (nb + 1) / 2;
  const size_t bytes = (size_t)N * cplx_bytes;
  const int slots = std::max(1, std::min(16, nb) * std::min(8, m));
  Layout L;
  size_t off = 0;
  L.phiA = off; off += align_up(bytes * (size_t)std::max(m, 1));
  L.phiB = off; off += align_up(bytes * (size_t)std::max(m, 1));
  L.acc = off;
  L.w = off; off += align_up(bytes * (size_t)slots);
  L.epart = off;
  L.tile_e = off;
  L.k0 = off; off += align_up(sizeof(double));
  L.gbpart = off; off += align_up(sizeof(double) * kGbParts);
  L.total = off;
  return L;
}

// k-mesh jobs: every set's real-space orbitals stay resident; one
// accumulator block; tile partials for every (k <= k') block.
Layout layout_kmesh(long long N, int cplx_bytes, int ngroups, int nk, int nbmax) {
  const int tc = tile_cap(nbmax, cplx_bytes);
  const size_t nb = (size_t)N * cplx_bytes;
  const int ntb = tile_count(nbmax, cplx_bytes);
  const int ntiles = (nk * (nk + 1) / 2) * ntb * ntb;
  // tile_e also holds the per-band partials of the energy taken from the gradient
  const int nparts = ntiles > nk * nbmax ? ntiles : nk * nbmax;
  Layout L;
  size_t off = 0;
  L.phiA = off; off += align_up(nb * (size_t)nbmax * nk);
  // gradient accumulators of every k-point: one transform per pair feeds the
  // blocks (k, k') and (k', k)
  L.phiB = off; off += align_up(nb * (size_t)nbmax * nk);
  L.acc = off; off += align_up(nb * (size_t)tc);
  L.w = off; off += align_up(nb * (size_t)tc * tc);
  L.epart = off; off += align_up(sizeof(double) * (size_t)tc * tc * ngroups);
  L.tile_e = off; off += align_up(sizeof(double) * (size_t)nparts);
  L.k0 = off; off += align_up(sizeof(double));
  L.gbpart = off; off += align_up(sizeof(double) * kGbParts);
  L.total = off;
  return L;
}

fock_status check_orbs(const fock_orbs* o, int npw, const char* name) {
  if (!o) return fail(FOCK_E_ARG, std::string(name) + " is NULL");
  if (o->nb < 0) return fail(FOCK_E_ARG, std::string(name) + ".nb < 0");
  if (o->nb > 0) {
    if (!o->c) return fail(FOCK_E_ARG, std::string(name) + ".c is NULL");
    if (!o->w) return fail(FOCK_E_ARG, std::string(name) + ".w is NULL");
    if (o->ld < npw) return fail(FOCK_E_ARG, std::string(name) + ".ld < npw");
  }
  return FOCK_OK;
}

#define FX_HIP(call)                                                                           \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) return fail(FOCK_E_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
struct Engine {
  const Plan& P;
  hipStream_t s;
  int ngroups;
  Engine(const Plan& p, hipStream_t st) : P(p), s(st) {
    ngroups = P.n[1] * P.n[2] / pencil_columns(P.n[0], (int)sizeof(T));
  }

  fock_status to_real_space(const void* c, int ld, int nb, void* box) {
    if (nb <= 0) return FOCK_OK;
    {
      FX_TRACE(KC_A1_SCATTER);
      FX_HIP(launch_zero<T>(box, P.N * nb, s));
      FX_HIP(launch_scatter<T>(c, ld, P.d_slot, P.npw, nb, box, P.N, s));
    }
    return transform(box, nb, +1);
  }

  fock_status transform(void* box, int nb, int sign) {
    PencilArgs pa{};
    pa.x = box;
    pa.tw1 = P.d_tw[0];
    pa.N = P.N;
    pa.n2 = P.n[1];
    pa.n3 = P.n[2];
    pa.count = nb;
    PlaneArgs la{};
    la.x = box;
    la.tw2 = P.d_tw[1];
    la.tw3 = P.d_tw[2];
    la.N = P.N;
    la.n1 = P.n[0];
    la.nb = nb;
    if (sign > 0) {
      { FX_TRACE(KC_A1_PENCIL); FX_HIP(launch_pencil<T>(PENCIL_INV, P.n[0], pa, nb * ngroups, s)); }
      { FX_TRACE(KC_A1_PLANE); FX_HIP(launch_plane<T>(PLANE_INV, P.n[1], P.n[2], la, nb * P.n[0], s)); }
    } else {
      { FX_TRACE(KC_A7_PLANE); FX_HIP(launch_plane<T>(PLANE_FWD, P.n[1], P.n[2], la, nb * P.n[0], s)); }
      { FX_TRACE(KC_A7_PENCIL); FX_HIP(launch_pencil<T>(PENCIL_FWD, P.n[0], pa, nb * ngroups, s)); }
    }
    return FOCK_OK;
  }

  KernelParams kparams(const double q[3], bool q_zero, const fock_cell* cell, double* d_k0) {
    KernelParams kp{};
    std::memcpy(kp.b, P.b, sizeof(kp.b));
    for (int k = 0; k < 3; ++k) kp.q[k] = q[k];
    kp.ecut = cell->ecut_fock;
    kp.k0 = d_k0;
    kp.q_zero = q_zero ? 1 : 0;
    return kp;
  }

  // K at q + G = 0 into d_k0 (device FP64 scalar).
  fock_status g0_constant(const fock_cell* cell, bool q_zero, double* d_k0, double* d_part) {
    if (!q_zero || cell->g0 == FOCK_G0_ZERO) {
      FX_HIP(launch_set_scalar(d_k0, 0.0, s));
      return FOCK_OK;
    }
    KernelParams kp{};
    std::memcpy(kp.b, P.b, sizeof(kp.b));
    const int nqt = cell->nq[0] * cell->nq[1] * cell->nq[2];
    const double head = nqt * P.omega / std::sqrt(kPi * cell->gb_alpha);
    FX_HIP(launch_gb(kp, P.n, cell->nq, cell->gb_alpha, head, d_part, kGbParts, d_k0, s));
    return FOCK_OK;
  }

  PlaneArgs plane_args(const void* phiA, const void* phiB, void* w, void* acc, const double* f, int i0, int j0,
                       int ti, int tj) {
    PlaneArgs la{};
    la.a = phiA;
    la.bsrc = phiB;
    la.w = w;
    la.acc = acc;
    la.f = f;
    la.tw2 = P.d_tw[1];
    la.tw3 = P.d_tw[2];
    la.N = P.N;
    la.i0 = i0;
    la.j0 = j0;
    la.ti = ti;
    la.tj = tj;
    la.n1 = P.n[0];
    la.fscale = 1.0;
    return la;
  }

  // P1 and P2 of one pair tile (energy: P2 only accumulates partials).
  // masked_reader: every pass that reads this pair buffer after P2 masks the
  // dead columns, so P2 need not write their zeros.
  fock_status tile_forward(const PlaneArgs& la, const KernelParams& kp, bool energy, double* epart,
                           int p1_mode, bool masked_reader) {
    const int tt = !la.tri ? la.ti * la.tj : p1_mode == PLANE_PAIR_FWD_G ? gtri_prefix(la.ti, la.tj) : tri_slot(0, la.ti);
    {
      FX_TRACE(KC_P1);
      FX_HIP(launch_plane<T>(p1_mode, P.n[1], P.n[2], la, tt * P.n[0], s));
    }
    PencilArgs pa{};
    pa.live = la.live;
    pa.x = la.w;
    pa.epart = energy ? epart : nullptr;
    pa.tw1 = P.d_tw[0];
    pa.kp = kp;
    pa.N = P.N;
    pa.n2 = P.n[1];
    pa.n3 = P.n[2];
    pa.count = tt;
    pa.skip_dead = masked_reader ? 1 : 0;
    if (energy) {
      FX_TRACE(KC_P2E);
      FX_HIP(launch_pencil<T>(PENCIL_FE, P.n[0], pa, tt * ngroups, s));
    } else {
      FX_TRACE(KC_P2);
      FX_HIP(launch_pencil<T>(PENCIL_FKI, P.n[0], pa, tt * ngroups, s));
    }
    return FOCK_OK;
  }

  // acc[0..nj) (real space) -> forward FFT -> sphere rows j0.. of out, scaled.
  fock_status finish(void* acc, int nj, int j0, void* out, int ldo, double s0, const double* wout,
                     const double* gscale) {
    fock_status st = transform(acc, nj, -1);
    if (st != FOCK_OK) return st;
    char* o = static_cast<char*>(out) + (size_t)j0 * ldo * sizeof(cx<T>);
    FX_TRACE(KC_A7_GATHER);
    FX_HIP(launch_gather<T>(acc, P.N, P.d_slot, P.npw, nj, o, ldo, s0, wout, j0, gscale, s));
    return FOCK_OK;
  }

  // Symmetric-schedule variant (FOCK_SYM_SCHEDULE overrides the default):
  //   0  fused inverse FFT + MAC into acc_J, v_ij written back and streamed
  //      into acc_I by a second kernel;
  //   1  fully parallel in-place inverse FFT, then one MAC kernel for both
  //      halves (default for FP32, whose transforms are VALU-bound, and for
  //      FP64 planes from 72 points wide);
  //   2  fused inverse FFT + MAC into acc_J, and a second fused pass that
  //      recomputes v_ij and accumulates the mirror into acc_I: no write-back,
  //      one more transform (default for FP64 planes up to 64 points wide,
  //      which are HBM-bound).
  // The fused passes hold a plane of complex accumulators beside the plane
  // being transformed; from 72 points wide in FP64 that exceeds the register
  // budget and spills, and schedule 1 measured faster: 72^3 -18%, 96^3 -22%,
  // 96 x 96 x 128 -51% per apply (48^3 and 64^3: schedule 2 faster by 6-16%).
  int sym_schedule() const {
    const char* e = std::getenv("FOCK_SYM_SCHEDULE");
    const int env = e ? std::atoi(e) : -1;
    if (env >= 0 && env <= 2) return env;
    return sizeof(T) == 8 && P.n[2] <= 64 ? 2 : 1;
  }

  // Apply of an occupied block to a different target block (or at q != 0):
  //   0  fused inverse plane FFT + multiply-accumulate, one workgroup per
  //      (target, plane) looping over the occupied orbitals of the tile;
  //   1  in-place inverse plane FFT of every pair of the tile, then the
  //      streaming multiply-accumulate (forward half only).
  // The fused pass holds a plane of accumulators beside the plane being
  // transformed; in FP64 beyond 96 x 96 that spills heavily, and schedule 1
  // is faster there (96 x 96 x 128, 64 x 64 orbitals: 112 against 150 ms).
  // Elsewhere the fused pass wins by 5-37% (FP32 at every size, FP64 up to
  // 96 x 96), since it moves the pair buffer once instead of three times.
  int apply_schedule() const {
    const char* e = std::getenv("FOCK_APPLY_SCHEDULE");
    const int env = e ? std::atoi(e) : -1;
    if (env == 0 || env == 1) return env;
    return sizeof(T) == 8 && P.n[1] * P.n[2] > 96 * 96 ? 1 : 0;
  }

  // Live plane columns of the pair buffer (FOCK_PRUNE=0: every column).
  const signed char* live() const {
    const char* e = std::getenv("FOCK_PRUNE");
    return e && e[0] == '0' ? nullptr : P.d_live;
  }

  // Gamma tiles: 0 = fused inverse plane FFT + MAC passes (forward, then a
  // recomputing mirror); 1 = in-place inverse plane FFT of the tile, then one
  // streaming pass for both halves.  The fused passes hold a whole plane per
  // block; from 72-point-wide planes they spill (FP64) or lose occupancy
  // (FP32), and the streaming schedule is faster in both precisions.
  int gamma_schedule() const {
    const char* e = std::getenv("FOCK_GAMMA_SCHEDULE");
    const int env = e ? std::atoi(e) : -1;
    if (env == 0 || env == 1) return env;
    return std::max(P.n[1], P.n[2]) >= 72 ? 1 : 0;
  }

  // One band-pair job: occupied block A (real space, weights fA) against
  // target block B.  energy: per-tile FP64 partials into tile_e[tile_base..];
  // apply with acc_full == null: per-target-tile accumulators, each finished
  // into out; apply with acc_full: accumulate into acc_full[nB][N] (zeroed by
  // the caller, finished by the caller).  sym: A == B at q = 0, tiles I <= J
  // only, v_ji = conj(v_ij) supplies the mirrored pairs (needs acc_full).
  struct PairJob {
    const void* phiA = nullptr;
    const double* fA = nullptr;
    int nA = 0;
    const void* phiB = nullptr;
    const double* gB = nullptr;
    int nB = 0;
    bool sym = false, energy = false;
    double escale = 1.0;
    int tile_base = 0;
    void* acc_full = nullptr;
    void* out = nullptr;
    int ldo = 0;
    double s0 = 0.0;
    const double* wout = nullptr;
    const double* gscale = nullptr;
    // cross: apply only, A != B, both halves from one transform per pair: the
    // forward half into acc_full (targets B, weights fA), the mirror half
    // f_j psi_j conj(v_ij) into acc_mirror (the rows of A, weights fB).  Holds
    // when the block with the roles swapped has kernel K(-q + G): its v is
    // conj(v_ij) in real space.
    bool cross = false;
    void* acc_mirror = nullptr;
    const double* fB = nullptr;
  };

  fock_status pairs(const KernelParams& kp, char* ws, const Layout& L, const PairJob& J, int* ntiles) {
    const Tiles t = tiles_for(J.nA, J.nB, (int)sizeof(cx<T>));
    void* w = ws + L.w;
    double* epart = reinterpret_cast<double*>(ws + L.epart);
    double* tile_e = reinterpret_cast<double*>(ws + L.tile_e) + J.tile_base;
    const size_t box = (size_t)P.N * sizeof(cx<T>);
    fock_status st;
    int tile = 0;
    if (J.cross) {
      if (J.energy || J.sym || !J.acc_full || !J.acc_mirror || !J.fB || sym_schedule() == 0)
        return fail(FOCK_E_ARG, "internal: bad cross-block job");
      const int T0 = t.ti;  // the pair tile edge (tiles_for), or the whole block
      for (int j0 = 0; j0 < J.nB; j0 += T0) {
        const int tj = (J.nB - j0) < T0 ? (J.nB - j0) : T0;
        for (int i0 = 0; i0 < J.nA; i0 += T0) {
          const int ti = (J.nA - i0) < T0 ? (J.nA - i0) : T0;
          PlaneArgs la = plane_args(J.phiA, J.phiB, w, nullptr, J.fA, i0, j0, ti, tj);
          la.live = live();
          // schedule 2 reads the pairs in the fused passes (every column), else
          // the in-place inverse reads them (live columns only)
          if ((st = tile_forward(la, kp, false, nullptr, PLANE_PAIR_FWD, sym_schedule() != 2)) != FOCK_OK) return st;
          if (sym_schedule() == 2) {
            PlaneArgs lp = la;
            lp.acc = static_cast<char*>(J.acc_full) + (size_t)j0 * box;
            {
              FX_TRACE(KC_P3);
              FX_HIP(launch_plane<T>(PLANE_INV_MAC, P.n[1], P.n[2], lp, tj * P.n[0], s));
            }
            PlaneArgs lb = la;
            lb.f = J.fB;
            lb.acc = static_cast<char*>(J.acc_mirror) + (size_t)i0 * box;
            FX_TRACE(KC_P3B);
            FX_HIP(launch_plane<T>(PLANE_INV_MAC_MIR, P.n[1], P.n[2], lb, ti * P.n[0], s));
            continue;
          }
          {
            FX_TRACE(KC_P3);
            PlaneArgs lv = plane_args(nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0, 0, 0);
            lv.x = w;
            lv.live = live();
            lv.nb = ti * tj;
            FX_HIP(launch_plane<T>(PLANE_INV, P.n[1], P.n[2], lv, ti * tj * P.n[0], s));
          }
          MacArgs ma{};
          ma.w = w;
          ma.phi = J.phiA;
          ma.f = J.fA;
          ma.acc = J.acc_mirror;
          ma.phi_b = J.phiB;
          ma.f_b = J.fB;
          ma.acc_b = J.acc_full;
          ma.N = P.N;
          ma.i0 = i0;
          ma.j0 = j0;
          ma.ti = ti;
          ma.tj = tj;
          ma.mirror = 1;
          FX_TRACE(KC_P3B);
          FX_HIP(launch_mac_pair<T>(ma, s));
        }
      }
      return FOCK_OK;
    }
    if (!J.sym) {
      for (int j0 = 0; j0 < J.nB; j0 += t.tj) {
        const int tj = (J.nB - j0) < t.tj ? (J.nB - j0) : t.tj;
        void* acc = J.acc_full ? static_cast<void*>(static_cast<char*>(J.acc_full) + (size_t)j0 * box)
                               : static_cast<void*>(ws + L.acc);
        if (!J.energy && !J.acc_full) {
          FX_TRACE(KC_ZERO);
          FX_HIP(launch_zero<T>(acc, P.N * tj, s));
        }
        for (int i0 = 0; i0 < J.nA; i0 += t.ti, ++tile) {
          const int ti = (J.nA - i0) < t.ti ? (J.nA - i0) : t.ti;
          PlaneArgs la = plane_args(J.phiA, J.phiB, w, acc, J.fA, i0, j0, ti, tj);
          la.live = live();
          if ((st = tile_forward(la, kp, J.energy, epart, PLANE_PAIR_FWD, apply_schedule() == 1)) != FOCK_OK)
            return st;
          if (J.energy) {
            FX_TRACE(KC_REDUCE);
            FX_HIP(launch_energy_tile(epart, ngroups, J.fA, J.gB, i0, j0, ti, tj, 0, 0, J.escale, tile_e + tile, s));
          } else if (apply_schedule() == 1) {
            {
              FX_TRACE(KC_P3);
              PlaneArgs lv = plane_args(nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0, 0, 0);
              lv.x = w;
              lv.live = live();
              lv.nb = ti * tj;
              FX_HIP(launch_plane<T>(PLANE_INV, P.n[1], P.n[2], lv, ti * tj * P.n[0], s));
            }
            // acc holds the tile's targets from row 0: target jj at row jj
            MacArgs ma{};
            ma.w = w;
            ma.phi = J.phiA;
            ma.f = J.fA;
            ma.acc = acc;  // mirror half: not used
            ma.phi_b = J.phiB;
            ma.acc_b = acc;
            ma.N = P.N;
            ma.i0 = i0;
            ma.j0 = 0;
            ma.ti = ti;
            ma.tj = tj;
            ma.mirror = 0;
            FX_TRACE(KC_P3B);
            FX_HIP(launch_mac_pair<T>(ma, s));
          } else {
            FX_TRACE(KC_P3);
            FX_HIP(launch_plane<T>(PLANE_INV_MAC, P.n[1], P.n[2], la, tj * P.n[0], s));
          }
        }
        if (!J.energy && !J.acc_full &&
            (st = finish(acc, tj, j0, J.out, J.ldo, J.s0, J.wout, J.gscale)) != FOCK_OK)
          return st;
      }
      if (ntiles) *ntiles = tile;
      return FOCK_OK;
    }
    // symmetric schedule
    if (!J.energy && !J.acc_full) return fail(FOCK_E_ARG, "internal: symmetric apply needs full accumulators");
    const int T0 = t.ti;  // the pair tile edge (tiles_for), or the whole block
    void* acc_all = J.acc_full;
    const void* phiA = J.phiA;
    for (int j0 = 0; j0 < J.nB; j0 += T0) {
      const int tj = (J.nB - j0) < T0 ? (J.nB - j0) : T0;
      for (int i0 = 0; i0 <= j0; i0 += T0, ++tile) {
        const int ti = (J.nA - i0) < T0 ? (J.nA - i0) : T0;
        PlaneArgs la = plane_args(phiA, phiA, w, nullptr, J.fA, i0, j0, ti, tj);
        la.live = live();
        // diagonal tiles transform only the pairs ii <= jj: in an apply
        // (schedules 1 and 2) the mirror supplies the rest, in an energy the
        // reduction counts the off-diagonal pairs twice
        la.tri = i0 == j0 && ti == tj && (J.energy || sym_schedule() != 0);
        const int tt = la.tri ? tri_slot(0, ti) : ti * tj;
        if ((st = tile_forward(la, kp, J.energy, epart, PLANE_PAIR_FWD, sym_schedule() == 1)) != FOCK_OK) return st;
        if (J.energy) {
          FX_TRACE(KC_REDUCE);
          FX_HIP(launch_energy_tile(epart, ngroups, J.fA, J.gB, i0, j0, ti, tj, 1, la.tri, J.escale, tile_e + tile, s));
          continue;
        }
        if (sym_schedule() == 2) {
          // fused inverse plane FFT + multiply-accumulate into acc_J, and for
          // off-diagonal tiles a second fused pass that recomputes v_ij and
          // accumulates f_j phi_j conj(v_ij) into acc_I (no write-back of v).
          PlaneArgs lp = la;
          lp.acc = static_cast<char*>(acc_all) + (size_t)j0 * box;
          {
            FX_TRACE(KC_P3);
            FX_HIP(launch_plane<T>(PLANE_INV_MAC, P.n[1], P.n[2], lp, tj * P.n[0], s));
          }
          if (i0 != j0 || (la.tri && ti > 1)) {
            PlaneArgs lb = lp;
            lb.acc = static_cast<char*>(acc_all) + (size_t)i0 * box;
            FX_TRACE(KC_P3B);
            FX_HIP(launch_plane<T>(PLANE_INV_MAC_MIR, P.n[1], P.n[2], lb, ti * P.n[0], s));
          }
          continue;
        }
        if (sym_schedule() == 0) {
          // fused inverse plane FFT + multiply-accumulate into acc_J; off-diagonal
          // tiles leave v_ij in real space for the mirrored half.
          PlaneArgs lp = la;
          lp.acc = static_cast<char*>(acc_all) + (size_t)j0 * box;
          lp.store_v = i0 != j0;
          {
            FX_TRACE(KC_P3);
            FX_HIP(launch_plane<T>(PLANE_INV_MAC, P.n[1], P.n[2], lp, tj * P.n[0], s));
          }
          if (i0 != j0) {
            PlaneArgs lb = lp;
            lb.acc = static_cast<char*>(acc_all) + (size_t)i0 * box;
            FX_TRACE(KC_P3B);
            FX_HIP(launch_mac_conj<T>(lb, P.n[1] * P.n[2], ti * P.n[0], s));
          }
          continue;
        }
        {
          // inverse plane FFT of every pair of the tile, in place: v_ij in real space
          FX_TRACE(KC_P3);
          PlaneArgs lv = plane_args(nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0, 0, 0);
          lv.x = w;
          lv.live = live();
          lv.nb = tt;
          FX_HIP(launch_plane<T>(PLANE_INV, P.n[1], P.n[2], lv, tt * P.n[0], s));
        }
        MacArgs ma{};
        ma.w = w;
        ma.phi = phiA;
        ma.f = J.fA;
        ma.acc = acc_all;
        ma.phi_b = phiA;
        ma.f_b = J.fA;
        ma.acc_b = acc_all;
        ma.N = P.N;
        ma.i0 = i0;
        ma.j0 = j0;
        ma.ti = ti;
        ma.tj = tj;
        ma.mirror = i0 != j0 || la.tri;
        ma.tri = la.tri;
        FX_TRACE(KC_P3B);
        FX_HIP(launch_mac_pair<T>(ma, s));
      }
    }
    if (ntiles) *ntiles = tile;
    return FOCK_OK;
  }
};


template <typename T>
fock_status apply_impl(const fock_cell* cell, const Plan& P, const double q[3], bool q_zero, const fock_orbs* occ,
                       const fock_orbs* tgt, char* ws, const Layout& L, hipStream_t s, void* out, double s0,
                       const double* wout, const double* gscale) {
  Engine<T> E(P, s);
  if (tgt->nb == 0) return FOCK_OK;
  double* d_k0 = reinterpret_cast<double*>(ws + L.k0);
  fock_status st = E.g0_constant(cell, q_zero, d_k0, reinterpret_cast<double*>(ws + L.gbpart));
  if (st != FOCK_OK) return st;
  void* phiA = ws + L.phiA;
  void* phiB = ws + L.phiB;
  const bool same = occ->c == tgt->c && occ->nb == tgt->nb && occ->ld == tgt->ld;
  if ((st = E.to_real_space(occ->c, occ->ld, occ->nb, phiA)) != FOCK_OK) return st;
  if (same) phiB = phiA;
  else if ((st = E.to_real_space(tgt->c, tgt->ld, tgt->nb, phiB)) != FOCK_OK) return st;
  typename Engine<T>::PairJob J;
  J.phiA = phiA;
  J.fA = occ->w;
  J.nA = occ->nb;
  J.phiB = phiB;
  J.gB = tgt->w;
  J.nB = tgt->nb;
  J.sym = same && q_zero && occ->nb > 0;
  J.out = out;
  J.ldo = tgt->ld;
  J.s0 = s0;
  J.wout = wout;
  J.gscale = gscale;
  if (J.sym || occ->nb == 0) {
    // every target accumulates in the (then unused) phiB region; finished once
    J.acc_full = ws + L.phiB;
    {
      FX_TRACE_S(KC_ZERO);
      FX_HIP(launch_zero<T>(J.acc_full, P.N * tgt->nb, s));
    }
    if (occ->nb > 0 && (st = E.pairs(E.kparams(q, q_zero, cell, d_k0), ws, L, J, nullptr)) != FOCK_OK) return st;
    return E.finish(J.acc_full, tgt->nb, 0, out, tgt->ld, occ->nb > 0 ? s0 : 0.0, wout, gscale);
  }
  return E.pairs(E.kparams(q, q_zero, cell, d_k0), ws, L, J, nullptr);
}

// Gamma point, real orbitals: V_x applied to the block itself, two real
// targets packed per complex transform.  Packed tiles: 16 real occupied x 8
// packed targets (16 real); only tiles that hold a pair i <= j run.
constexpr int kGammaTi = 16, kGammaTj = 8;
static_assert(kGammaTi <= kMacTile, "the streaming Gamma MAC holds one tile row per thread");

template <typename T>
fock_status apply_gamma_impl(const fock_cell* cell, const Plan& P, const fock_orbs* o, char* ws, const Layout& L,
                             hipStream_t s, void* out, double s0) {
  Engine<T> E(P, s);
  const int n = o->nb, m = (n + 1) / 2;
  if (n == 0) return FOCK_OK;
  const double q0[3] = {0.0, 0.0, 0.0};
  double* d_k0 = reinterpret_cast<double*>(ws + L.k0);
  fock_status st = E.g0_constant(cell, true, d_k0, reinterpret_cast<double*>(ws + L.gbpart));
  if (st != FOCK_OK) return st;
  void* pk = ws + L.phiA;   // packed orbitals in real space [m][N]
  void* acc = ws + L.phiB;  // packed accumulators [m][N]
  const size_t box = (size_t)P.N * sizeof(cx<T>);
  {
    FX_TRACE(KC_A1_SCATTER);
    FX_HIP(launch_zero<T>(pk, P.N * m, s));
    FX_HIP(launch_scatter_pack<T>(o->c, o->ld, P.d_slot, P.npw, n, pk, P.N, s));
  }
  if ((st = E.transform(pk, m, +1)) != FOCK_OK) return st;
  {
    FX_TRACE_S(KC_ZERO);
    FX_HIP(launch_zero<T>(acc, P.N * m, s));
  }
  const KernelParams kp = E.kparams(q0, true, cell, d_k0);
  for (int j0 = 0; j0 < m; j0 += kGammaTj) {
    const int tj = std::min(kGammaTj, m - j0);
    for (int i0 = 0; i0 < n && i0 <= 2 * (j0 + tj) - 1; i0 += kGammaTi) {
      const int ti = std::min(kGammaTi, n - i0);
      PlaneArgs la = E.plane_args(pk, pk, ws + L.w, nullptr, o->w, i0, j0, ti, tj);
      la.live = E.live();
      la.nreal = n;
      // diagonal tile (the occupied reals of the packed targets): only the
      // pairs with a non-zero weight, i <= 2q + 1, are transformed
      la.tri = i0 == 2 * j0;
      const int tt = la.tri ? gtri_prefix(ti, tj) : ti * tj;
      // both Gamma schedules mask the dead columns when they read the pairs
      if ((st = E.tile_forward(la, kp, false, nullptr, PLANE_PAIR_FWD_G, true)) != FOCK_OK) return st;
      if (E.gamma_schedule() == 1) {
        {
          FX_TRACE(KC_P3);
          PlaneArgs lv = E.plane_args(nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0, 0, 0);
          lv.x = ws + L.w;
          lv.live = E.live();
          lv.nb = tt;
          FX_HIP(launch_plane<T>(PLANE_INV, P.n[1], P.n[2], lv, tt * P.n[0], s));
        }
        MacArgs ma{};
        ma.w = ws + L.w;
        ma.phi = pk;
        ma.f = o->w;
        ma.acc = acc;
        ma.N = P.N;
        ma.i0 = i0;
        ma.j0 = j0;
        ma.ti = ti;
        ma.tj = tj;
        ma.tri = la.tri;
        FX_TRACE(KC_P3B);
        FX_HIP(launch_mac_gamma<T>(ma, n, s));
        continue;
      }
      PlaneArgs lp = la;
      lp.acc = static_cast<char*>(acc) + (size_t)j0 * box;
      {
        FX_TRACE(KC_P3);
        FX_HIP(launch_plane<T>(PLANE_INV_MAC_G, P.n[1], P.n[2], lp, tj * P.n[0], s));
      }
      PlaneArgs lb = la;
      lb.acc = static_cast<char*>(acc) + (size_t)(i0 / 2) * box;
      {
        FX_TRACE(KC_P3B);
        FX_HIP(launch_plane<T>(PLANE_INV_MAC_MIR_G, P.n[1], P.n[2], lb, ti * P.n[0], s));
      }
    }
  }
  if ((st = E.transform(acc, m, -1)) != FOCK_OK) return st;
  FX_TRACE(KC_A7_GATHER);
  FX_HIP(launch_gather_unpack<T>(acc, P.N, P.d_slot, P.npw, P.n, n, out, o->ld, s0, s));
  return FOCK_OK;
}

template <typename T>
fock_status energy_impl(const fock_cell* cell, const Plan& P, const double q[3], bool q_zero, const fock_orbs* occ,
                        const fock_orbs* tgt, char* ws, const Layout& L, hipStream_t s, double* ex) {
  Engine<T> E(P, s);
  if (occ->nb == 0 || tgt->nb == 0) {
    FX_HIP(launch_set_scalar(ex, 0.0, s));
    return FOCK_OK;
  }
  double* d_k0 = reinterpret_cast<double*>(ws + L.k0);
  fock_status st = E.g0_constant(cell, q_zero, d_k0, reinterpret_cast<double*>(ws + L.gbpart));
  if (st != FOCK_OK) return st;
  void* phiA = ws + L.phiA;
  void* phiB = ws + L.phiB;
  const bool same = occ->c == tgt->c && occ->nb == tgt->nb && occ->ld == tgt->ld;
  if ((st = E.to_real_space(occ->c, occ->ld, occ->nb, phiA)) != FOCK_OK) return st;
  if (same) phiB = phiA;
  else if ((st = E.to_real_space(tgt->c, tgt->ld, tgt->nb, phiB)) != FOCK_OK) return st;
  typename Engine<T>::PairJob J;
  J.phiA = phiA;
  J.fA = occ->w;
  J.nA = occ->nb;
  J.phiB = phiB;
  J.gB = tgt->w;
  J.nB = tgt->nb;
  J.sym = same && q_zero;
  J.energy = true;
  int ntiles = 0;
  if ((st = E.pairs(E.kparams(q, q_zero, cell, d_k0), ws, L, J, &ntiles)) != FOCK_OK) return st;
  const double scale = -0.5 / (P.omega * (double)P.N * (double)P.N);
  FX_HIP(launch_energy_final(reinterpret_cast<double*>(ws + L.tile_e), ntiles, scale, ex, s));
  return FOCK_OK;
}

struct Prepared {
  std::shared_ptr<Plan> plan;
  Layout L;
  bool q_zero = false;
};

fock_status check_cell_host(const fock_cell* cell, int dtype) {
  if (!cell) return fail(FOCK_E_ARG, "cell is NULL");
  if (dtype != FOCK_C128 && dtype != FOCK_C64) return fail(FOCK_E_ARG, "dtype must be FOCK_C128 or FOCK_C64");
  for (int k = 0; k < 3; ++k)
    if (cell->n[k] <= 0) return fail(FOCK_E_ARG, "grid sizes must be positive");
  if (cell->npw <= 0 || !cell->miller) return fail(FOCK_E_ARG, "empty G-sphere (npw <= 0 or miller NULL)");
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      if (!std::isfinite(cell->a[i][j])) return fail(FOCK_E_ARG, "lattice vectors must be finite");
  return FOCK_OK;
}

// Exactness of the pair products on the grid (reduced exchange cutoff).
// With M_a the largest |m_a| of the sphere, a pair density has Fourier
// components only at |m_a| <= 2 M_a, and K(q+G) is non-zero only inside the
// ball |q+G|^2 <= E_fock, whose points have |m_a| <= F_a(q).  The grid
// transform of the product adds to the component at m the true components at
// m + n t (t != 0), so rho(G) is exact wherever K != 0 when
// n_a - F_a > 2 M_a.  The product phi * v then has components up to
// M_a + min(F_a, 2 M_a), and nothing lands on the sphere (|m_a| <= M_a) when
// n_a > min(F_a, 2 M_a) + 2 M_a: the same condition.  F_a is bounded by
// (|a_a| sqrt(E_fock) + |a_a . q|) / (2 pi), since m_a = a_a . (q+G) / (2 pi)
// - a_a . q / (2 pi); without a cutoff (E_fock <= 0) F_a is unbounded and the
// rule is n_a >= 4 M_a + 1.  need[a] receives the smallest admissible n_a.
void alias_need(const fock_cell* cell, const double* q, int nq, int need[3]) {
  int M[3] = {0, 0, 0};
  for (int p = 0; p < cell->npw; ++p)
    for (int k = 0; k < 3; ++k) {
      const int m = std::abs(cell->miller[3 * p + k]);
      M[k] = m > M[k] ? m : M[k];
    }
  for (int k = 0; k < 3; ++k) {
    const double* ak = cell->a[k];
    const double alen = std::sqrt(ak[0] * ak[0] + ak[1] * ak[1] + ak[2] * ak[2]);
    long long F = 2LL * M[k];
    if (cell->ecut_fock > 0.0) {
      double fq = 0.0;
      for (int j = 0; j < (nq > 0 ? nq : 1); ++j) {
        const double* qj = nq > 0 ? q + 3 * j : nullptr;
        const double aq = qj ? std::fabs(ak[0] * qj[0] + ak[1] * qj[1] + ak[2] * qj[2]) : 0.0;
        fq = std::max(fq, (alen * std::sqrt(cell->ecut_fock) + aq) / (2.0 * kPi));
      }
      // a hair of slack so that a ball touching a lattice point counts it
      const long long Fk = (long long)std::floor(fq + 1e-9);
      F = std::min(F, Fk);
    }
    need[k] = (int)(F + 2LL * M[k] + 1);
  }
}

fock_status check_alias(const fock_cell* cell, const double* q, int nq) {
  int need[3];
  alias_need(cell, q, nq, need);
  for (int k = 0; k < 3; ++k)
    if (cell->n[k] < need[k]) {
      char buf[200];
      std::snprintf(buf, sizeof buf,
                    "grid n=%d on axis %d is below %d, the smallest without aliasing for this sphere, cutoff and q",
                    cell->n[k], k, need[k]);
      return fail(FOCK_E_ALIAS, buf);
    }
  return FOCK_OK;
}

// q + G = 0 for a non-zero q means q is a reciprocal-lattice vector:
// its fractional coordinates a_a . q / (2 pi) are all integers.
fock_status check_q(const fock_cell* cell, const double q[3], bool* q_zero) {
  if (!q) return fail(FOCK_E_ARG, "q is NULL");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(q[k])) return fail(FOCK_E_ARG, "q must be finite");
  *q_zero = q[0] == 0.0 && q[1] == 0.0 && q[2] == 0.0;
  if (!*q_zero) {
    bool all_int = true;
    for (int k = 0; k < 3; ++k) {
      const double s = (cell->a[k][0] * q[0] + cell->a[k][1] * q[1] + cell->a[k][2] * q[2]) / (2.0 * kPi);
      if (std::fabs(s - std::nearbyint(s)) > 1e-9) all_int = false;
    }
    if (all_int) return fail(FOCK_E_SINGULAR_Q, "q is a non-zero reciprocal-lattice vector: fold it into the zone");
  }
  return FOCK_OK;
}

fock_status prepare(const fock_cell* cell, const double q[3], int dtype, const fock_orbs* occ, const fock_orbs* tgt,
                    void* ws, size_t ws_bytes, Prepared* out) {
  fock_status st = check_cell_host(cell, dtype);
  if (st != FOCK_OK) return st;
  if (!grid_supported(cell->n, dtype))
    return fail(FOCK_E_UNSUPPORTED_GRID, "no compiled transforms for grid " + grid_str(cell->n));
  if ((st = check_orbs(occ, cell->npw, "occ")) != FOCK_OK) return st;
  if ((st = check_orbs(tgt, cell->npw, "tgt")) != FOCK_OK) return st;
  if ((st = check_q(cell, q, &out->q_zero)) != FOCK_OK) return st;
  if ((st = check_alias(cell, q, 1)) != FOCK_OK) return st;
  const long long N = (long long)cell->n[0] * cell->n[1] * cell->n[2];
  const int ngroups = cell->n[1] * cell->n[2] / pencil_columns(cell->n[0], tbytes_of(dtype));
  out->L = layout(N, dtype == FOCK_C128 ? 16 : 8, ngroups, occ->nb, tgt->nb);
  if (!ws || ws_bytes < out->L.total) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, out->L.total);
    return fail(FOCK_E_WORKSPACE, buf);
  }
  return get_plan(cell, dtype, &out->plan);
}

// Exchange energy over a k-point mesh and its gradient.  Block (k, k')
// pairs targets at k with occupied orbitals at k', q = k - k'.
// ex_from_grad (with ex and grad, grad_ex null): no energy pass; after the
// gradient, E = 1/2 Re sum_k sum_j <c_jk | dE/d conj(c_jk)>.
template <typename T>
fock_status kmesh_impl(const fock_cell* cell, const Plan& P, int nk, const double* kpts, const fock_orbs* sets,
                       char* ws, const Layout& L, hipStream_t s, double* ex, const double* grad_ex,
                       void* const* grad, bool ex_from_grad = false) {
  Engine<T> E(P, s);
  const size_t box = (size_t)P.N * sizeof(cx<T>);
  int nbmax = 0;
  for (int k = 0; k < nk; ++k) nbmax = sets[k].nb > nbmax ? sets[k].nb : nbmax;
  double* d_k0 = reinterpret_cast<double*>(ws + L.k0);
  fock_status st = E.g0_constant(cell, true, d_k0, reinterpret_cast<double*>(ws + L.gbpart));
  if (st != FOCK_OK) return st;
  auto phi = [&](int k) { return static_cast<void*>(ws + L.phiA + (size_t)k * nbmax * box); };
  for (int k = 0; k < nk; ++k)
    if ((st = E.to_real_space(sets[k].c, sets[k].ld, sets[k].nb, phi(k))) != FOCK_OK) return st;
  auto qof = [&](int kt, int ko, double q[3]) {
    for (int a = 0; a < 3; ++a) q[a] = kpts[3 * kt + a] - kpts[3 * ko + a];
    return q[0] == 0.0 && q[1] == 0.0 && q[2] == 0.0;
  };
  if (ex && !ex_from_grad) {
    // E_kk' = E_k'k: blocks k <= k' only, off-diagonal ones counted twice
    int base = 0;
    for (int k = 0; k < nk; ++k) {
      for (int kp = k; kp < nk; ++kp) {
        if (sets[k].nb == 0 || sets[kp].nb == 0) continue;
        double q[3];
        const bool qz = qof(k, kp, q);
        typename Engine<T>::PairJob J;
        J.phiA = phi(kp);
        J.fA = sets[kp].w;
        J.nA = sets[kp].nb;
        J.phiB = phi(k);
        J.gB = sets[k].w;
        J.nB = sets[k].nb;
        J.sym = kp == k;
        J.energy = true;
        J.escale = kp == k ? 1.0 : 2.0;
        J.tile_base = base;
        int nt = 0;
        if ((st = E.pairs(E.kparams(q, qz, cell, d_k0), ws, L, J, &nt)) != FOCK_OK) return st;
        base += nt;
      }
    }
    const double scale = -0.5 / (P.omega * (double)P.N * (double)P.N);
    FX_HIP(launch_energy_final(reinterpret_cast<double*>(ws + L.tile_e), base, scale, ex, s));
  }
  if (grad) {
    // dE/d conj(c_jk) = w_jk sum_k' (V_x with occupied set k', q = k - k') psi_jk.
    // The block (k', k) has q' = -q and K(q' + G) = K(q - G), so its
    // real-space v is conj of block (k, k')'s: every pair of a block k < k'
    // is transformed once and feeds both gradients (schedules 1 and 2).
    auto acc = [&](int k) { return static_cast<void*>(ws + L.phiB + (size_t)k * nbmax * box); };
    const double s0 = -1.0 / (P.omega * (double)P.N * (double)P.N);
    const bool cross = E.sym_schedule() != 0;
    for (int k = 0; k < nk; ++k) {
      if (sets[k].nb == 0 || !grad[k]) continue;
      FX_TRACE_S(KC_ZERO);
      FX_HIP(launch_zero<T>(acc(k), P.N * sets[k].nb, s));
    }
    auto job = [&](int kt, int ko) {
      typename Engine<T>::PairJob J;
      J.phiA = phi(ko);
      J.fA = sets[ko].w;
      J.nA = sets[ko].nb;
      J.phiB = phi(kt);
      J.gB = sets[kt].w;
      J.nB = sets[kt].nb;
      J.sym = ko == kt;
      J.acc_full = acc(kt);
      return J;
    };
    for (int k = 0; k < nk; ++k) {
      for (int kp = k; kp < nk; ++kp) {
        if (sets[k].nb == 0 || sets[kp].nb == 0) continue;
        const bool gk = grad[k] != nullptr, gkp = grad[kp] != nullptr;
        double q[3];
        if (kp == k || !cross || !(gk && gkp)) {
          // one direction at a time: (k, kp) into k, and (kp, k) into kp
          if (gk) {
            const bool qz = qof(k, kp, q);
            if ((st = E.pairs(E.kparams(q, qz, cell, d_k0), ws, L, job(k, kp), nullptr)) != FOCK_OK) return st;
          }
          if (kp != k && gkp) {
            const bool qz = qof(kp, k, q);
            if ((st = E.pairs(E.kparams(q, qz, cell, d_k0), ws, L, job(kp, k), nullptr)) != FOCK_OK) return st;
          }
          continue;
        }
        // targets at k, occupied at kp; the mirror half goes to the targets at kp
        const bool qz = qof(k, kp, q);
        typename Engine<T>::PairJob J = job(k, kp);
        J.cross = true;
        J.acc_mirror = acc(kp);
        J.fB = sets[k].w;
        if ((st = E.pairs(E.kparams(q, qz, cell, d_k0), ws, L, J, nullptr)) != FOCK_OK) return st;
      }
    }
    for (int k = 0; k < nk; ++k) {
      if (sets[k].nb == 0 || !grad[k]) continue;
      if ((st = E.finish(acc(k), sets[k].nb, 0, grad[k], sets[k].ld, s0, sets[k].w, grad_ex)) != FOCK_OK) return st;
    }
  }
  if (ex && ex_from_grad) {
    double* part = reinterpret_cast<double*>(ws + L.tile_e);
    int off = 0;
    for (int k = 0; k < nk; ++k) {
      if (sets[k].nb == 0) continue;
      FX_TRACE(KC_REDUCE);
      FX_HIP(launch_band_dot<T>(sets[k].c, sets[k].ld, grad[k], sets[k].ld, P.npw, nullptr, sets[k].nb, part + off, s));
      off += sets[k].nb;
    }
    if (off == 0) {
      FX_HIP(launch_set_scalar(ex, 0.0, s));
    } else {
      FX_HIP(launch_energy_final(part, off, 0.5, ex, s));
    }
  }
  return FOCK_OK;
}

fock_status kmesh_prepare(const fock_cell* cell, int32_t nk, const double* kpts, int32_t dtype, const fock_orbs* sets,
                          void* ws, size_t ws_bytes, std::shared_ptr<Plan>* plan, Layout* L) {
  fock_status st = check_cell_host(cell, dtype);
  if (st != FOCK_OK) return st;
  if (!grid_supported(cell->n, dtype))
    return fail(FOCK_E_UNSUPPORTED_GRID, "no compiled transforms for grid " + grid_str(cell->n));
  if (nk <= 0 || !kpts || !sets) return fail(FOCK_E_ARG, "need nk > 0, kpts and sets");
  int nbmax = 0;
  for (int k = 0; k < nk; ++k) {
    if ((st = check_orbs(&sets[k], cell->npw, "sets[k]")) != FOCK_OK) return st;
    nbmax = sets[k].nb > nbmax ? sets[k].nb : nbmax;
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(kpts[3 * k + a])) return fail(FOCK_E_ARG, "k-points must be finite");
  }
  for (int k = 0; k < nk; ++k)
    for (int kp = 0; kp < nk; ++kp) {
      const double q[3] = {kpts[3 * k] - kpts[3 * kp], kpts[3 * k + 1] - kpts[3 * kp + 1],
                           kpts[3 * k + 2] - kpts[3 * kp + 2]};
      bool qz;
      if ((st = check_q(cell, q, &qz)) != FOCK_OK) return st;
      if ((st = check_alias(cell, q, 1)) != FOCK_OK) return st;
    }
  const long long N = (long long)cell->n[0] * cell->n[1] * cell->n[2];
  const int ngroups = cell->n[1] * cell->n[2] / pencil_columns(cell->n[0], tbytes_of(dtype));
  *L = layout_kmesh(N, dtype == FOCK_C128 ? 16 : 8, ngroups, nk, nbmax);
  if (!ws || ws_bytes < L->total) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, L->total);
    return fail(FOCK_E_WORKSPACE, buf);
  }
  return get_plan(cell, dtype, plan);
}


// ---------------------------------------------------------------------------
// Band loops of the Car-Parrinello code: charge density and the force of the
// local Hamiltonian, one 3-D transform per band, bands taken in chunks.
// ---------------------------------------------------------------------------
constexpr int kBandChunk = 64;   // bands per chunk of launches
constexpr int kBandGroups = 8;   // band groups per plane: workgroups = n1 * kBandGroups

struct BandLayout {
  size_t box, part, total;
  int cb;
};

BandLayout band_layout(long long N, int cplx_bytes, int nb) {
  BandLayout L{};
  L.cb = nb < kBandChunk ? (nb > 0 ? nb : 1) : kBandChunk;
  size_t off = 0;
  L.box = off; off += align_up((size_t)L.cb * N * cplx_bytes);
  L.part = off; off += align_up(sizeof(double) * (size_t)kBandGroups * N);
  L.total = off;
  return L;
}

fock_status band_prepare(const fock_cell* cell, int32_t dtype, const fock_orbs* orbs, void* ws, size_t ws_bytes,
                         std::shared_ptr<Plan>* plan, BandLayout* L) {
  fock_status st = check_cell_host(cell, dtype);
  if (st != FOCK_OK) return st;
  if (!grid_supported(cell->n, dtype))
    return fail(FOCK_E_UNSUPPORTED_GRID, "no compiled transforms for grid " + grid_str(cell->n));
  if ((st = check_orbs(orbs, cell->npw, "orbs")) != FOCK_OK) return st;
  const long long N = (long long)cell->n[0] * cell->n[1] * cell->n[2];
  *L = band_layout(N, dtype == FOCK_C128 ? 16 : 8, orbs->nb);
  if (!ws || ws_bytes < L->total) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, L->total);
    return fail(FOCK_E_WORKSPACE, buf);
  }
  return get_plan(cell, dtype, plan);
}

// rho[r] = sum_b w_b |psi_b(r)|^2, psi_b(r) = Omega^{-1/2} sum_G c_b(G) e^{iG.r}
template <typename T>
fock_status band_density_impl(const Plan& P, const fock_orbs* o, double* rho, char* ws, const BandLayout& L,
                              hipStream_t s) {
  Engine<T> E(P, s);
  void* box = ws + L.box;
  double* part = reinterpret_cast<double*>(ws + L.part);
  for (int b0 = 0; b0 < o->nb; b0 += L.cb) {
    const int n = std::min(L.cb, o->nb - b0);
    const char* c = static_cast<const char*>(o->c) + (size_t)b0 * o->ld * sizeof(cx<T>);
    {
      FX_TRACE(KC_A1_SCATTER);
      FX_HIP(launch_zero<T>(box, P.N * n, s));
      FX_HIP(launch_scatter<T>(c, o->ld, P.d_slot, P.npw, n, box, P.N, s));
    }
    PencilArgs pa{};
    pa.x = box;
    pa.tw1 = P.d_tw[0];
    pa.N = P.N;
    pa.n2 = P.n[1];
    pa.n3 = P.n[2];
    pa.count = n;
    { FX_TRACE(KC_A1_PENCIL); FX_HIP(launch_pencil<T>(PENCIL_INV, P.n[0], pa, n * E.ngroups, s)); }
    PlaneArgs la{};
    la.x = box;
    la.tw2 = P.d_tw[1];
    la.tw3 = P.d_tw[2];
    la.N = P.N;
    la.n1 = P.n[0];
    la.nb = n;
    la.f = o->w;
    la.i0 = b0;
    la.fscale = 1.0 / P.omega;
    la.ngrp = kBandGroups;
    la.part = part;
    la.accumulate = b0 > 0;
    { FX_TRACE(KC_BAND_DENS); FX_HIP(launch_plane<T>(PLANE_DENS, P.n[1], P.n[2], la, P.n[0] * kBandGroups, s)); }
  }
  FX_TRACE(KC_REDUCE);
  FX_HIP(launch_group_sum(part, o->nb > 0 ? kBandGroups : 0, P.N, rho, s));
  return FOCK_OK;
}

// out_b(G) = -w_b (1/2 |k+G|^2 c_b(G) + (V psi_b)(G)),
// (V psi)(G) = N^{-1} sum_r V(r) psi~(r) e^{-iG.r}, psi~ = sum_G c(G) e^{iG.r}
template <typename T>
fock_status band_force_impl(const Plan& P, const double k[3], const fock_orbs* o, const void* vloc, void* out,
                            char* ws, const BandLayout& L, hipStream_t s) {
  Engine<T> E(P, s);
  void* box = ws + L.box;
  for (int b0 = 0; b0 < o->nb; b0 += L.cb) {
    const int n = std::min(L.cb, o->nb - b0);
    const char* c = static_cast<const char*>(o->c) + (size_t)b0 * o->ld * sizeof(cx<T>);
    {
      FX_TRACE(KC_A1_SCATTER);
      FX_HIP(launch_zero<T>(box, P.N * n, s));
      FX_HIP(launch_scatter<T>(c, o->ld, P.d_slot, P.npw, n, box, P.N, s));
    }
    PencilArgs pa{};
    pa.x = box;
    pa.tw1 = P.d_tw[0];
    pa.N = P.N;
    pa.n2 = P.n[1];
    pa.n3 = P.n[2];
    pa.count = n;
    { FX_TRACE(KC_A1_PENCIL); FX_HIP(launch_pencil<T>(PENCIL_INV, P.n[0], pa, n * E.ngroups, s)); }
    PlaneArgs la{};
    la.x = box;
    la.tw2 = P.d_tw[1];
    la.tw3 = P.d_tw[2];
    la.N = P.N;
    la.n1 = P.n[0];
    la.nb = n;
    la.ngrp = kBandGroups;
    la.vloc = vloc;
    { FX_TRACE(KC_BAND_VMUL); FX_HIP(launch_plane<T>(PLANE_VMUL, P.n[1], P.n[2], la, P.n[0] * kBandGroups, s)); }
    { FX_TRACE(KC_A7_PENCIL); FX_HIP(launch_pencil<T>(PENCIL_FWD, P.n[0], pa, n * E.ngroups, s)); }
    ForceArgs fa{};
    fa.box = box;
    fa.N = P.N;
    fa.slot = P.d_slot;
    fa.npw = P.npw;
    fa.c = o->c;
    fa.ldc = o->ld;
    fa.out = out;
    fa.ldo = o->ld;
    fa.w = o->w;
    fa.j0 = b0;
    std::memcpy(fa.b, P.b, sizeof(fa.b));
    for (int a = 0; a < 3; ++a) fa.k[a] = k[a];
    fa.n1 = P.n[0];
    fa.n2 = P.n[1];
    fa.n3 = P.n[2];
    { FX_TRACE(KC_BAND_GATHER); FX_HIP(launch_force_gather<T>(fa, n, s)); }
  }
  return FOCK_OK;
}

// ---------------------------------------------------------------------------
// Batched form: several systems, one persistent launch inside one hipGraph.
// ---------------------------------------------------------------------------
struct BatchPlanImpl {
  int device = 0, dtype = 0, nsys = 0, cus = 0;
  std::vector<std::shared_ptr<Plan>> plans;
  std::vector<fock_cell> cells;
  std::vector<fock_orbs> orbs;  // occupied blocks
  std::vector<fock_orbs> tgt;   // target blocks
  std::vector<double> q;        // [nsys][3]
  std::vector<char> qzero;
  bool persistent_ok = true;    // every system one block applied to itself at q = 0 on a cubic grid
  std::vector<void*> outs;      // plan-owned [tgt.nb][tgt.ld] results
  double* d_ex = nullptr;       // [nsys] energies
  double* d_bandE = nullptr;    // per-band energy terms, systems one after another
  std::vector<int> band_off;
  std::vector<void*> phi, acc;
  std::vector<void*> allocs;
  double* d_k0 = nullptr;
  double* d_gbpart = nullptr;
  BatchSys* d_sys = nullptr;
  BatchSeg* d_seg = nullptr;
  void** d_slots = nullptr;
  unsigned long long* d_ticket = nullptr;
  int* d_done = nullptr;
  int* d_abort = nullptr;
  long long* d_wait = nullptr;  // bound on one dependency wait of the persistent kernel, wall-clock ticks
  double wait_khz = 0.0;        // wall-clock ticks per millisecond
  double wait_ms = 0.0;         // the plan's own bound (fock_batch_set_wait_limit with ms <= 0 restores it)
  std::vector<void*> slot_mem;
  size_t slot_bytes = 0;
  int nseg = 0;
  long long total_units = 0;
  long long pairs = 0;
  BatchParams prm;
  const char* prm_source = "default";  // how prm was chosen: default, tuned now, or read from the tune cache
  // mode 1: the systems are split over `branches` independent graph branches
  // (each its own stream while capturing), each with a workspace sized for
  // its largest system
  std::vector<void*> kws;
  std::vector<size_t> kws_bytes;
  std::vector<hipStream_t> branch_streams;  // capture streams of branches 1.. (branch 0: cap)
  std::vector<hipEvent_t> branch_events;    // fork and join events (no timing)
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::string info;
  ~BatchPlanImpl() {
    (void)hipSetDevice(device);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (void* p : allocs) (void)hipFree(p);
    for (hipEvent_t e : branch_events) (void)hipEventDestroy(e);
    for (hipStream_t st : branch_streams) (void)hipStreamDestroy(st);
    if (cap) (void)hipStreamDestroy(cap);
  }
  fock_status alloc(void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes > 0 ? bytes : 1);
    if (e != hipSuccess) return fail(FOCK_E_HIP, std::string("batch allocation: ") + hipGetErrorString(e));
    allocs.push_back(*p);
    return FOCK_OK;
  }
};

// A dependency wait of the persistent kernel lasts, in a correct schedule, at
// most until the running blocks finish the units they hold (tickets are
// handed out in dependency order): milliseconds.  The bound is 1 s, or four
// times the tuned replay if that is longer, so a scheduling fault ends the
// launch with FOCK_E_HIP from fock_batch_check instead of a long hang.
constexpr double kBatchWaitMs = 1000.0;

fock_status batch_set_wait(BatchPlanImpl& B, double ms) {
  if (!B.d_wait) return FOCK_OK;
  const long long ticks = std::max(1LL, (long long)std::llround(ms * B.wait_khz));
  FX_HIP(hipMemcpy(B.d_wait, &ticks, sizeof ticks, hipMemcpyHostToDevice));
  return FOCK_OK;
}

// Builds the unit list: system-interleaved pair tiles (per system: target tile
// outer, occupied tile I <= J inner, the order of the single-system symmetric
// schedule), emitted in pipelined rounds P1(r), P2(r-1), P3(r-2), MAC(r-3).
void batch_segments(const BatchPlanImpl& B, const BatchParams& prm, std::vector<BatchSeg>* out, long long* total) {
  struct TileRef {
    int sys, i0, j0, ti, tj;
  };
  std::vector<std::vector<TileRef>> per(B.nsys);
  for (int s = 0; s < B.nsys; ++s) {
    const int nb = B.orbs[s].nb, T = prm.tile;
    for (int j0 = 0; j0 < nb; j0 += T)
      for (int i0 = 0; i0 <= j0; i0 += T)
        per[s].push_back({s, i0, j0, std::min(T, nb - i0), std::min(T, nb - j0)});
  }
  std::vector<TileRef> tiles;
  for (size_t k = 0;; ++k) {
    bool any = false;
    for (int s = 0; s < B.nsys; ++s)
      if (k < per[s].size()) {
        tiles.push_back(per[s][k]);
        any = true;
      }
    if (!any) break;
  }
  const int nt = (int)tiles.size();
  std::vector<int> seg_of(4 * (size_t)nt, -1);
  std::vector<int> prev_same(nt, -1), last(B.nsys, -1);
  for (int r = 0; r < nt; ++r) {
    prev_same[r] = last[tiles[r].sys];
    last[tiles[r].sys] = r;
  }
  out->clear();
  long long start = 0;
  for (int round = 0; round < nt + 3; ++round) {
    for (int stage = 0; stage < 4; ++stage) {
      const int r = round - stage;
      if (r < 0 || r >= nt) continue;
      const TileRef& t = tiles[r];
      const Plan& P = *B.plans[t.sys];
      const int n = P.n[0];
      const int ngroups = n * n / pencil_columns(n, tbytes_of(B.dtype));
      BatchSeg g{};
      g.start = start;
      g.sys = t.sys;
      g.stage = stage;
      g.slot = r % prm.slots;
      g.i0 = t.i0;
      g.j0 = t.j0;
      g.ti = t.ti;
      g.tj = t.tj;
      g.dep[0] = g.dep[1] = -1;
      const int tt = t.ti * t.tj;
      switch (stage) {
        case BS_P1:
          g.units = tt * n;
          if (r >= prm.slots) g.dep[0] = seg_of[4 * (r - prm.slots) + BS_MAC];
          break;
        case BS_P2:
          g.units = tt * ngroups;
          g.dep[0] = seg_of[4 * r + BS_P1];
          break;
        case BS_P3:
          g.units = tt * n;
          g.dep[0] = seg_of[4 * r + BS_P2];
          break;
        default:
          g.units = (int)((P.N + kBatchW - 1) / kBatchW);
          g.dep[0] = seg_of[4 * r + BS_P3];
          if (prev_same[r] >= 0) g.dep[1] = seg_of[4 * prev_same[r] + BS_MAC];
          break;
      }
      seg_of[4 * r + stage] = (int)out->size();
      out->push_back(g);
      start += g.units;
    }
  }
  *total = start;
}

// E_s = 1/2 sum_j g_j Re <psi_j | V_x psi_j> per system, from the results on
// the sphere (the reciprocal-space energy of the block: for V_x built from the
// occupied block with its occupations, <psi_j|V_x psi_j> = -Omega sum_i f_i
// sum_G K |rho_ij(G)|^2).  Two fixed-order stages.
template <typename T>
fock_status batch_energies(BatchPlanImpl& B, hipStream_t s) {
  for (int k = 0; k < B.nsys; ++k) {
    const fock_orbs& t = B.tgt[k];
    if (t.nb == 0) {
      FX_HIP(launch_set_scalar(B.d_ex + k, 0.0, s));
      continue;
    }
    double* part = B.d_bandE + B.band_off[k];
    FX_HIP(launch_band_dot<T>(t.c, t.ld, B.outs[k], t.ld, B.plans[k]->npw, t.w, t.nb, part, s));
    FX_HIP(launch_energy_final(part, t.nb, 0.5, B.d_ex + k, s));
  }
  return FOCK_OK;
}

template <typename T>
fock_status batch_capture(BatchPlanImpl& B, const BatchParams& prm) {
  if (prm.mode == 0 && !B.persistent_ok) return fail(FOCK_E_ARG, "internal: persistent schedule not applicable");
  // the previous graph is dropped first
  if (B.exec) {
    (void)hipGraphExecDestroy(B.exec);
    B.exec = nullptr;
  }
  if (B.graph) {
    (void)hipGraphDestroy(B.graph);
    B.graph = nullptr;
  }
  fock_status st;
  long long total = 0;
  BatchArgs a{};
  int occ = 1, bpc = 0, grid = 0;
  if (prm.mode == 0) {
    // scheduler tables (re-allocated per schedule)
    std::vector<BatchSeg> segs;
    batch_segments(B, prm, &segs, &total);
    B.nseg = (int)segs.size();
    B.total_units = total;
    void* p = nullptr;
    if ((st = B.alloc(&p, sizeof(BatchSeg) * segs.size())) != FOCK_OK) return st;
    B.d_seg = static_cast<BatchSeg*>(p);
    if ((st = B.alloc(&p, sizeof(int) * segs.size())) != FOCK_OK) return st;
    B.d_done = static_cast<int*>(p);
    FX_HIP(hipMemcpy(B.d_seg, segs.data(), sizeof(BatchSeg) * segs.size(), hipMemcpyHostToDevice));
    a.sys = B.d_sys;
    a.seg = B.d_seg;
    a.nseg = B.nseg;
    a.total_units = total;
    a.units_per_ticket = prm.units_per_ticket;
    a.slots = B.d_slots;
    a.ticket = B.d_ticket;
    a.done = B.d_done;
    a.abort_flag = B.d_abort;
    a.wait_ticks = B.d_wait;
    occ = prm.blocks_per_cu >= 2 ? 2 : 1;
    const int bpc_max = batch_blocks_per_cu<T>(occ);
    bpc = prm.blocks_per_cu > 0 && prm.blocks_per_cu < bpc_max ? prm.blocks_per_cu : bpc_max;
    grid = bpc * B.cus;
  }
  std::vector<int> branch_of;
  if (prm.mode == 1) {
    // systems to branches: longest first onto the least loaded branch, the
    // load of a system taken as its pairs times N log N
    const int nbr = std::max(1, std::min(prm.branches, B.nsys));
    std::vector<int> order(B.nsys);
    std::vector<double> cost(B.nsys), load(nbr, 0.0);
    for (int k = 0; k < B.nsys; ++k) {
      order[k] = k;
      const double N = (double)B.plans[k]->N;
      cost[k] = (double)B.orbs[k].nb * (double)B.tgt[k].nb * N * std::log2(N);
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    branch_of.assign(B.nsys, 0);
    for (int k : order) {
      const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      branch_of[k] = b;
      load[b] += cost[k];
    }
    // one workspace per branch, sized for its largest system (kept across captures)
    std::vector<size_t> need(nbr, 0);
    for (int k = 0; k < B.nsys; ++k) {
      const Plan& P = *B.plans[k];
      const int ng = P.n[1] * P.n[2] / pencil_columns(P.n[0], (int)sizeof(T));
      need[branch_of[k]] = std::max(need[branch_of[k]], layout(P.N, (int)sizeof(cx<T>), ng, B.orbs[k].nb,
                                                                B.tgt[k].nb).total);
    }
    for (int b = 0; b < nbr; ++b) {
      if ((int)B.kws.size() <= b) {
        B.kws.push_back(nullptr);
        B.kws_bytes.push_back(0);
      }
      if (B.kws_bytes[b] < need[b]) {
        void* p = nullptr;
        if ((st = B.alloc(&p, need[b])) != FOCK_OK) return st;
        B.kws[b] = p;
        B.kws_bytes[b] = need[b];
      }
    }
    while ((int)B.branch_streams.size() < nbr - 1) {
      hipStream_t bs = nullptr;
      FX_HIP(hipStreamCreateWithFlags(&bs, hipStreamNonBlocking));
      B.branch_streams.push_back(bs);
    }
    while ((int)B.branch_events.size() < nbr) {
      hipEvent_t ev = nullptr;
      FX_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      B.branch_events.push_back(ev);
    }
  }
  // capture; tracing events must not enter the graph
  Tracer& TR = tracer();
  const bool tr_on = TR.on;
  TR.on = false;
  hipStream_t s = B.cap;
  auto body = [&]() -> fock_status {
    if (prm.mode == 1) {
      // each system's own per-shape schedule (the single-system path); the
      // systems of one branch in turn, the branches forked from and joined
      // back into the capture stream (independent paths of the graph)
      const int nbr = (int)std::min(B.kws.size(), (size_t)std::max(1, std::min(prm.branches, B.nsys)));
      std::vector<hipStream_t> bst(nbr, s);
      for (int b = 1; b < nbr; ++b) bst[b] = B.branch_streams[b - 1];
      if (nbr > 1) {
        FX_HIP(hipEventRecord(B.branch_events[0], s));
        for (int b = 1; b < nbr; ++b) FX_HIP(hipStreamWaitEvent(bst[b], B.branch_events[0], 0));
      }
      for (int k = 0; k < B.nsys; ++k) {
        const Plan& P = *B.plans[k];
        const int b = branch_of[k];
        const int ng = P.n[1] * P.n[2] / pencil_columns(P.n[0], (int)sizeof(T));
        const Layout L = layout(P.N, (int)sizeof(cx<T>), ng, B.orbs[k].nb, B.tgt[k].nb);
        if (L.total > B.kws_bytes[b]) return fail(FOCK_E_WORKSPACE, "batch workspace too small");
        const double s0 = -1.0 / (P.omega * (double)P.N * (double)P.N);
        fock_status st2 = apply_impl<T>(&B.cells[k], P, &B.q[3 * k], B.qzero[k] != 0, &B.orbs[k], &B.tgt[k],
                                        static_cast<char*>(B.kws[b]), L, bst[b], B.outs[k], s0, nullptr, nullptr);
        if (st2 != FOCK_OK) return st2;
      }
      for (int b = 1; b < nbr; ++b) {
        FX_HIP(hipEventRecord(B.branch_events[b], bst[b]));
        FX_HIP(hipStreamWaitEvent(s, B.branch_events[b], 0));
      }
      return batch_energies<T>(B, s);
    }
    FX_HIP(launch_batch_reset(B.d_ticket, B.d_done, B.nseg, B.d_abort, s));
    for (int k = 0; k < B.nsys; ++k) {
      Engine<T> E(*B.plans[k], s);
      fock_status st2 = E.g0_constant(&B.cells[k], true, B.d_k0 + k, B.d_gbpart);
      if (st2 != FOCK_OK) return st2;
      if ((st2 = E.to_real_space(B.orbs[k].c, B.orbs[k].ld, B.orbs[k].nb, B.phi[k])) != FOCK_OK) return st2;
      FX_HIP(launch_zero<T>(B.acc[k], B.plans[k]->N * B.orbs[k].nb, s));
    }
    FX_HIP(launch_batch<T>(a, occ, grid, s));
    for (int k = 0; k < B.nsys; ++k) {
      const Plan& P = *B.plans[k];
      Engine<T> E(P, s);
      const double s0 = -1.0 / (P.omega * (double)P.N * (double)P.N);
      fock_status st2 = E.finish(B.acc[k], B.orbs[k].nb, 0, B.outs[k], B.orbs[k].ld, s0, nullptr, nullptr);
      if (st2 != FOCK_OK) return st2;
    }
    return batch_energies<T>(B, s);
  };
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    TR.on = tr_on;
    return fail(FOCK_E_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
  }
  st = body();
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(s, &g);
  TR.on = tr_on;
  if (st != FOCK_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(FOCK_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  B.graph = g;
  FX_HIP(hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0));
  char buf[256];
  if (prm.mode == 1)
    std::snprintf(buf, sizeof buf,
                  "{\"mode\": \"kernels\", \"branches\": %d, \"systems\": %d, \"pairs\": %lld, \"ms\": %.4f, "
                  "\"source\": \"%s\"}",
                  std::max(1, std::min(prm.branches, B.nsys)), B.nsys, B.pairs, prm.ms, B.prm_source);
  else
    std::snprintf(buf, sizeof buf,
                  "{\"mode\": \"persistent\", \"tile\": %d, \"slots\": %d, \"units_per_ticket\": %d, "
                  "\"blocks_per_cu\": %d, \"grid\": %d, \"segments\": %d, \"units\": %lld, \"pairs\": %lld, "
                  "\"ms\": %.4f, \"source\": \"%s\"}",
                  prm.tile, prm.slots, prm.units_per_ticket, bpc, grid, B.nseg, total, B.pairs, prm.ms, B.prm_source);
  B.info = buf;
  return FOCK_OK;
}

std::string batch_signature(const BatchPlanImpl& B) {
  hipDeviceProp_t prop{};
  (void)hipGetDeviceProperties(&prop, B.device);
  std::string key = std::string(prop.gcnArchName) + "|cu" + std::to_string(B.cus) + "|" +
                    (B.dtype == FOCK_C128 ? "c128" : "c64");
  for (int k = 0; k < B.nsys; ++k)
    key += "|" + std::to_string(B.plans[k]->n[0]) + ":" + std::to_string(B.orbs[k].nb);
  for (char& ch : key)
    if (ch == '"' || ch == '\\' || ch == ' ') ch = '_';
  return key;
}

template <typename T>
fock_status batch_time(BatchPlanImpl& B, double* ms) {
  hipEvent_t a = nullptr, b = nullptr;
  FX_HIP(hipEventCreate(&a));
  FX_HIP(hipEventCreate(&b));
  hipError_t e = hipGraphLaunch(B.exec, B.cap);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(a, B.cap);
  if (e == hipSuccess) e = hipGraphLaunch(B.exec, B.cap);
  if (e == hipSuccess) e = hipEventRecord(b, B.cap);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float t = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return fail(FOCK_E_HIP, std::string("batch timing: ") + hipGetErrorString(e));
  int aborted = 0;
  FX_HIP(hipMemcpy(&aborted, B.d_abort, sizeof(int), hipMemcpyDeviceToHost));
  if (aborted) return fail(FOCK_E_HIP, "batch scheduler aborted a dependency wait");
  *ms = t;
  return FOCK_OK;
}

// Autotuner: times the candidate schedules on this batch and keeps the fastest.
template <typename T>
fock_status batch_tune_and_capture(BatchPlanImpl& B, const std::string& cache) {
  const std::string key = batch_signature(B);
  BatchParams best;
  const char* env = std::getenv("FOCK_BATCH_TUNE");
  const bool tune = !(env && std::atoi(env) == 0);
  // FOCK_BATCH_MODE = 0 / 1 restricts the plan to one mode (no cache use)
  const char* me = std::getenv("FOCK_BATCH_MODE");
  int force_mode = me && (std::atoi(me) == 0 || std::atoi(me) == 1) ? std::atoi(me) : -1;
  if (!B.persistent_ok) force_mode = 1;  // only the per-shape schedules apply
  if (!tune) {
    // untuned: the default schedule; FOCK_BATCH_TICKET sets the units per ticket
    best.mode = force_mode == 1 ? 1 : 0;
    if (const char* tk = std::getenv("FOCK_BATCH_TICKET")) {
      const int v = std::atoi(tk);
      if (v >= 1 && v <= (1 << 20)) best.units_per_ticket = v;
    }
    if (const char* nb = std::getenv("FOCK_BATCH_BRANCHES")) {
      const int v = std::atoi(nb);
      if (v >= 1 && v <= kBatchMaxBranches) best.branches = v;
    }
  } else if (force_mode < 0 && tune_cache_lookup(cache, key, &best)) {
    B.prm_source = "tune cache";
  } else {
    B.prm_source = "tuned";
    std::map<std::tuple<int, int, int>, double> seen;
    auto eval = [&](int tile, int upt, int bpc, double* ms) -> fock_status {
      auto k = std::make_tuple(tile, upt, bpc);
      auto it = seen.find(k);
      if (it != seen.end()) {
        *ms = it->second;
        return FOCK_OK;
      }
      BatchParams p;
      p.tile = tile;
      p.units_per_ticket = upt;
      p.blocks_per_cu = bpc;
      fock_status st = batch_capture<T>(B, p);
      if (st != FOCK_OK) return st;
      if ((st = batch_time<T>(B, ms)) != FOCK_OK) return st;
      if (const char* lg = std::getenv("FOCK_TUNE_LOG"); lg && std::atoi(lg) != 0)
        std::fprintf(stderr, "[fock tune] tile %d ticket %d blocks/CU %d: %.3f ms\n", tile, upt, bpc, *ms);
      seen[k] = *ms;
      return FOCK_OK;
    };
    fock_status st;
    double best_ms = -1.0;
    if (force_mode != 1) {
      // persistent kernel: greedy coordinate search over (tile, units per ticket, blocks per CU)
      const std::vector<int> tiles = {16, 8};
      const std::vector<int> tickets = {128, 32, 512};
      std::vector<int> bpcs = {1};
      if (batch_blocks_per_cu<T>(2) >= 2) bpcs.push_back(2);
      int cur[3] = {tiles[0], tickets[0], bpcs[0]};
      if ((st = eval(cur[0], cur[1], cur[2], &best_ms)) != FOCK_OK) return st;
      const std::vector<int>* axes[3] = {&tiles, &tickets, &bpcs};
      for (int pass = 0; pass < 2; ++pass) {
        bool moved = false;
        for (int ax = 0; ax < 3; ++ax) {
          for (int v : *axes[ax]) {
            int trial[3] = {cur[0], cur[1], cur[2]};
            trial[ax] = v;
            double ms = 0.0;
            if ((st = eval(trial[0], trial[1], trial[2], &ms)) != FOCK_OK) return st;
            if (ms < best_ms) {
              best_ms = ms;
              cur[ax] = v;
              moved = true;
            }
          }
        }
        if (!moved) break;
      }
      best.tile = cur[0];
      best.units_per_ticket = cur[1];
      best.blocks_per_cu = cur[2];
      best.ms = best_ms;
      best.mode = 0;
    }
    if (force_mode != 0) {
      // the per-shape kernels of every system in one graph, on 1 .. 4 branches
      for (int nbr = 1; nbr <= std::min(kBatchMaxBranches, B.nsys); ++nbr) {
        BatchParams p;
        p.mode = 1;
        p.branches = nbr;
        double ms = 0.0;
        if ((st = batch_capture<T>(B, p)) != FOCK_OK) return st;
        if ((st = batch_time<T>(B, &ms)) != FOCK_OK) return st;
        if (const char* lg = std::getenv("FOCK_TUNE_LOG"); lg && std::atoi(lg) != 0)
          std::fprintf(stderr, "[fock tune] per-shape kernels on %d branch(es): %.3f ms\n", nbr, ms);
        if (best_ms < 0.0 || ms < best_ms) {
          best = p;
          best.ms = ms;
          best_ms = ms;
        }
      }
    }
    if (force_mode < 0) tune_cache_store(cache, key, best);
  }
  B.prm = best;
  B.wait_ms = std::max(kBatchWaitMs, 4.0 * best.ms);
  fock_status st = batch_set_wait(B, B.wait_ms);
  if (st != FOCK_OK) return st;
  return batch_capture<T>(B, best);
}

template <typename T>
fock_status batch_create(BatchPlanImpl& B, const std::string& cache) {
  const size_t cb = sizeof(cx<T>);
  fock_status st;
  void* p = nullptr;
  // plan-owned results and energies (both schedules)
  int nbands = 0;
  for (int k = 0; k < B.nsys; ++k) {
    const fock_orbs& t = B.tgt[k];
    if ((st = B.alloc(&p, cb * (size_t)t.nb * (size_t)t.ld)) != FOCK_OK) return st;
    B.outs.push_back(p);
    B.band_off.push_back(nbands);
    nbands += t.nb;
    B.pairs += (long long)B.orbs[k].nb * t.nb;
  }
  if ((st = B.alloc(&p, sizeof(double) * B.nsys)) != FOCK_OK) return st;
  B.d_ex = static_cast<double*>(p);
  if ((st = B.alloc(&p, sizeof(double) * (size_t)std::max(nbands, 1))) != FOCK_OK) return st;
  B.d_bandE = static_cast<double*>(p);
  if ((st = B.alloc(&p, sizeof(int))) != FOCK_OK) return st;
  B.d_abort = static_cast<int*>(p);
  FX_HIP(hipMemset(B.d_abort, 0, sizeof(int)));
  if ((st = B.alloc(&p, sizeof(long long))) != FOCK_OK) return st;
  B.d_wait = static_cast<long long*>(p);
  int khz = 0;
  FX_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, B.device));
  B.wait_khz = khz > 0 ? (double)khz : 1.0e5;
  B.wait_ms = kBatchWaitMs;
  if ((st = batch_set_wait(B, B.wait_ms)) != FOCK_OK) return st;
  FX_HIP(hipStreamCreateWithFlags(&B.cap, hipStreamNonBlocking));
  if (!B.persistent_ok) return batch_tune_and_capture<T>(B, cache);
  // the persistent kernel's state
  long long nmax = 0;
  for (int k = 0; k < B.nsys; ++k) {
    const Plan& P = *B.plans[k];
    nmax = P.N > nmax ? P.N : nmax;
    void *ph = nullptr, *ac = nullptr;
    if ((st = B.alloc(&ph, cb * P.N * (size_t)B.orbs[k].nb)) != FOCK_OK) return st;
    if ((st = B.alloc(&ac, cb * P.N * (size_t)B.orbs[k].nb)) != FOCK_OK) return st;
    B.phi.push_back(ph);
    B.acc.push_back(ac);
  }
  if ((st = B.alloc(&p, sizeof(double) * B.nsys)) != FOCK_OK) return st;
  B.d_k0 = static_cast<double*>(p);
  if ((st = B.alloc(&p, sizeof(double) * kGbParts)) != FOCK_OK) return st;
  B.d_gbpart = static_cast<double*>(p);
  std::vector<BatchSys> sys(B.nsys);
  for (int k = 0; k < B.nsys; ++k) {
    const Plan& P = *B.plans[k];
    BatchSys& S = sys[k];
    S.phi = B.phi[k];
    S.acc = B.acc[k];
    S.f = B.orbs[k].w;
    S.tw = P.d_tw[0];
    std::memcpy(S.kp.b, P.b, sizeof(S.kp.b));
    S.kp.q[0] = S.kp.q[1] = S.kp.q[2] = 0.0;
    S.kp.ecut = B.cells[k].ecut_fock;
    S.kp.k0 = B.d_k0 + k;
    S.kp.q_zero = 1;
    S.N = P.N;
    S.n = P.n[0];
    S.nb = B.orbs[k].nb;
    S.ngroups = P.n[1] * P.n[2] / pencil_columns(P.n[0], (int)sizeof(T));
  }
  if ((st = B.alloc(&p, sizeof(BatchSys) * B.nsys)) != FOCK_OK) return st;
  B.d_sys = static_cast<BatchSys*>(p);
  FX_HIP(hipMemcpy(B.d_sys, sys.data(), sizeof(BatchSys) * B.nsys, hipMemcpyHostToDevice));
  // pair buffers: sized for the largest tile of the largest grid
  B.slot_bytes = cb * (size_t)nmax * kMacTile * kMacTile;
  for (int k = 0; k < kBatchSlots; ++k) {
    if ((st = B.alloc(&p, B.slot_bytes)) != FOCK_OK) return st;
    B.slot_mem.push_back(p);
  }
  if ((st = B.alloc(&p, sizeof(void*) * kBatchSlots)) != FOCK_OK) return st;
  B.d_slots = static_cast<void**>(p);
  FX_HIP(hipMemcpy(B.d_slots, B.slot_mem.data(), sizeof(void*) * kBatchSlots, hipMemcpyHostToDevice));
  if ((st = B.alloc(&p, sizeof(unsigned long long))) != FOCK_OK) return st;
  B.d_ticket = static_cast<unsigned long long*>(p);
  return batch_tune_and_capture<T>(B, cache);
}
// ---------------------------------------------------------------------------
// Allocation-free apply (fock_apply_noalloc): the plan's device tables and
// the workspace of fock_apply live in one fixed device array per GPU.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = FOCK_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// One copy per GPU, held until the process ends.  Host code never uses this
// name as an address: the device address comes from hipGetSymbolAddress,
// per device (scratch_base).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Device address of the current GPU's scratch array, looked up once per
// device with that device current.
fock_status scratch_base(char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(FOCK_E_HIP, "no HIP device available");
  if (dev < 0 || dev >= kMaxDevices) return fail(FOCK_E_HIP, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(FOCK_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<char*>(g_scratch_ptr[dev]);
  return FOCK_OK;
}

// Scratch layout of one call: slot table, live-column table, three twiddle
// tables, then the workspace of fock_apply.
struct ScratchLayout {
  size_t slot, live, tw[3], ws, total;
};
ScratchLayout scratch_layout(const fock_cell* cell, int dtype, const Layout& L) {
  const size_t cb = dtype == FOCK_C128 ? 16 : 8;
  ScratchLayout S;
  size_t off = 0;
  S.slot = off; off += align_up(sizeof(int32_t) * (size_t)cell->npw);
  S.live = off; off += align_up((size_t)cell->n[2]);
  for (int k = 0; k < 3; ++k) {
    S.tw[k] = off;
    off += align_up(cb * (size_t)cell->n[k]);
  }
  S.ws = off; off += L.total;
  S.total = off;
  return S;
}

template <typename T>
fock_status apply_noalloc_impl(const fock_cell* cell, const double q[3], const fock_orbs* occ, const fock_orbs* tgt,
                               void* vx_out, hipStream_t s) {
  const int dtype = sizeof(T) == 8 ? FOCK_C128 : FOCK_C64;
  double b[3][3], omega = 0.0;
  fock_status st = check_plan_cell(cell, dtype, b, &omega);
  if (st != FOCK_OK) return st;
  if ((st = check_orbs(occ, cell->npw, "occ")) != FOCK_OK) return st;
  if ((st = check_orbs(tgt, cell->npw, "tgt")) != FOCK_OK) return st;
  bool q_zero = false;
  if ((st = check_q(cell, q, &q_zero)) != FOCK_OK) return st;
  if ((st = check_alias(cell, q, 1)) != FOCK_OK) return st;
  if (tgt->nb > 0 && !vx_out) return fail(FOCK_E_ARG, "vx_out is NULL");
  const long long N = (long long)cell->n[0] * cell->n[1] * cell->n[2];
  const int ngroups = cell->n[1] * cell->n[2] / pencil_columns(cell->n[0], (int)sizeof(T));
  const Layout L = layout(N, (int)sizeof(cx<T>), ngroups, occ->nb, tgt->nb);
  const ScratchLayout S = scratch_layout(cell, dtype, L);
  if (S.total > kScratchBytes) {
    char buf[200];
    std::snprintf(buf, sizeof buf, "this call needs %zu bytes of device memory; the allocation-free scratch holds %zu",
                  S.total, kScratchBytes);
    return fail(FOCK_E_WORKSPACE, buf);
  }
  std::vector<int> slot;
  std::vector<signed char> live;
  bool has_live = false;
  if ((st = sphere_tables(cell, &slot, &live, &has_live)) != FOCK_OK) return st;
  char* base = nullptr;
  if ((st = scratch_base(&base)) != FOCK_OK) return st;
  // tables, rewritten by every call (stream ordered after the previous call's kernels)
  FX_HIP(launch_put_words(base + S.slot, slot.data(), sizeof(int32_t) * slot.size(), s));
  if (has_live) {
    live.resize((live.size() + 3) / 4 * 4, (signed char)-1);
    FX_HIP(launch_put_words(base + S.live, live.data(), live.size(), s));
  }
  for (int k = 0; k < 3; ++k) {
    const std::vector<unsigned char> tw = host_twiddles(cell->n[k], dtype);
    FX_HIP(launch_put_words(base + S.tw[k], tw.data(), tw.size(), s));
  }
  Plan P;
  P.owns = false;
  (void)hipGetDevice(&P.device);
  for (int k = 0; k < 3; ++k) P.n[k] = cell->n[k];
  P.N = N;
  P.dtype = dtype;
  std::memcpy(P.a, cell->a, sizeof(P.a));
  std::memcpy(P.b, b, sizeof(b));
  P.omega = omega;
  P.npw = cell->npw;
  P.d_slot = reinterpret_cast<int*>(base + S.slot);
  P.d_live = has_live ? reinterpret_cast<signed char*>(base + S.live) : nullptr;
  for (int k = 0; k < 3; ++k) P.d_tw[k] = base + S.tw[k];
  const double s0 = -1.0 / (omega * (double)N * (double)N);
  return apply_impl<T>(cell, P, q, q_zero, occ, tgt, base + S.ws, L, s, vx_out, s0, nullptr, nullptr);
}

}  // namespace

extern "C" {

fock_status fock_apply_noalloc(const fock_cell* cell, const double q[3], int32_t dtype, const fock_orbs* occ,
                               const fock_orbs* tgt, void* vx_out, void* stream) {
  if (dtype != FOCK_C128 && dtype != FOCK_C64) return fail(FOCK_E_ARG, "dtype must be FOCK_C128 or FOCK_C64");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dtype == FOCK_C128) return apply_noalloc_impl<double>(cell, q, occ, tgt, vx_out, s);
  return apply_noalloc_impl<float>(cell, q, occ, tgt, vx_out, s);
}

size_t fock_workspace_size(const fock_cell* cell, int32_t dtype, int32_t n_occ, int32_t n_tgt) {
  if (!cell || n_occ < 0 || n_tgt < 0 || (dtype != FOCK_C128 && dtype != FOCK_C64)) return 0;
  if (!grid_supported(cell->n, dtype)) return 0;
  const long long N = (long long)cell->n[0] * cell->n[1] * cell->n[2];
  const int ngroups = cell->n[1] * cell->n[2] / pencil_columns(cell->n[0], tbytes_of(dtype));
  return layout(N, dtype == FOCK_C128 ? 16 : 8, ngroups, n_occ, n_tgt).total;
}

fock_status fock_apply(const fock_cell* cell, const double q[3], int32_t dtype, const fock_orbs* occ,
                       const fock_orbs* tgt, void* vx_out, void* ws, size_t ws_bytes, void* stream) {
  Prepared pr;
  fock_status st = prepare(cell, q, dtype, occ, tgt, ws, ws_bytes, &pr);
  if (st != FOCK_OK) return st;
  if (tgt->nb > 0 && !vx_out) return fail(FOCK_E_ARG, "vx_out is NULL");
  const Plan& P = *pr.plan;
  const double s0 = -1.0 / (P.omega * (double)P.N * (double)P.N);
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  if (dtype == FOCK_C128)
    return apply_impl<double>(cell, P, q, pr.q_zero, occ, tgt, w, pr.L, s, vx_out, s0, nullptr, nullptr);
  return apply_impl<float>(cell, P, q, pr.q_zero, occ, tgt, w, pr.L, s, vx_out, s0, nullptr, nullptr);
}

size_t fock_workspace_size_gamma(const fock_cell* cell, int32_t dtype, int32_t nb) {
  if (!cell || nb < 0 || (dtype != FOCK_C128 && dtype != FOCK_C64)) return 0;
  if (!grid_supported(cell->n, dtype)) return 0;
  const long long N = (long long)cell->n[0] * cell->n[1] * cell->n[2];
  return layout_gamma(N, dtype == FOCK_C128 ? 16 : 8, nb).total;
}

fock_status fock_apply_gamma(const fock_cell* cell, int32_t dtype, const fock_orbs* orbs, void* vx_out, void* ws,
                             size_t ws_bytes, void* stream) {
  fock_status st = check_cell_host(cell, dtype);
  if (st != FOCK_OK) return st;
  if (!grid_supported(cell->n, dtype))
    return fail(FOCK_E_UNSUPPORTED_GRID, "no compiled transforms for grid " + grid_str(cell->n));
  if ((st = check_orbs(orbs, cell->npw, "orbs")) != FOCK_OK) return st;
  const double q0[3] = {0.0, 0.0, 0.0};
  if ((st = check_alias(cell, q0, 1)) != FOCK_OK) return st;
  if (orbs->nb > 0 && !vx_out) return fail(FOCK_E_ARG, "vx_out is NULL");
  const long long N = (long long)cell->n[0] * cell->n[1] * cell->n[2];
  const Layout L = layout_gamma(N, dtype == FOCK_C128 ? 16 : 8, orbs->nb);
  if (!ws || ws_bytes < L.total) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, L.total);
    return fail(FOCK_E_WORKSPACE, buf);
  }
  std::shared_ptr<Plan> P;
  if ((st = get_plan(cell, dtype, &P)) != FOCK_OK) return st;
  const double s0 = -1.0 / (P->omega * (double)P->N * (double)P->N);
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  if (dtype == FOCK_C128) return apply_gamma_impl<double>(cell, *P, orbs, w, L, s, vx_out, s0);
  return apply_gamma_impl<float>(cell, *P, orbs, w, L, s, vx_out, s0);
}

fock_status fock_energy(const fock_cell* cell, const double q[3], int32_t dtype, const fock_orbs* occ,
                        const fock_orbs* tgt, double* ex_out, void* ws, size_t ws_bytes, void* stream) {
  Prepared pr;
  fock_status st = prepare(cell, q, dtype, occ, tgt, ws, ws_bytes, &pr);
  if (st != FOCK_OK) return st;
  if (!ex_out) return fail(FOCK_E_ARG, "ex_out is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  if (dtype == FOCK_C128) return energy_impl<double>(cell, *pr.plan, q, pr.q_zero, occ, tgt, w, pr.L, s, ex_out);
  return energy_impl<float>(cell, *pr.plan, q, pr.q_zero, occ, tgt, w, pr.L, s, ex_out);
}

fock_status fock_energy_backward(const fock_cell* cell, const double q[3], int32_t dtype, const fock_orbs* occ,
                                 const fock_orbs* tgt, const double* grad_ex, void* grad_occ, void* grad_tgt,
                                 void* ws, size_t ws_bytes, void* stream) {
  Prepared pr;
  fock_status st = prepare(cell, q, dtype, occ, tgt, ws, ws_bytes, &pr);
  if (st != FOCK_OK) return st;
  if (!grad_ex) return fail(FOCK_E_ARG, "grad_ex is NULL");
  const Plan& P = *pr.plan;
  const double s0 = -0.5 / (P.omega * (double)P.N * (double)P.N);
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  if (grad_tgt) {
    // dE/d conj(d_j) = 1/2 g_j (V_x psi_j)
    st = dtype == FOCK_C128 ? apply_impl<double>(cell, P, q, pr.q_zero, occ, tgt, w, pr.L, s, grad_tgt, s0, tgt->w, grad_ex)
                            : apply_impl<float>(cell, P, q, pr.q_zero, occ, tgt, w, pr.L, s, grad_tgt, s0, tgt->w, grad_ex);
    if (st != FOCK_OK) return st;
  }
  // One block with equal weights at q = 0: the roles are symmetric and both
  // gradients are the same array (f_i V_x phi_i / 2); copy instead of a second apply.
  const bool same = occ->c == tgt->c && occ->nb == tgt->nb && occ->ld == tgt->ld && occ->w == tgt->w;
  if (grad_occ && grad_tgt && same && pr.q_zero) {
    if (grad_occ != grad_tgt && occ->nb > 0) {
      // rows of npw values at the leading dimension ld: padding columns are left alone
      const size_t eb = dtype == FOCK_C128 ? 16 : 8, pitch = (size_t)occ->ld * eb;
      FX_HIP(hipMemcpy2DAsync(grad_occ, pitch, grad_tgt, pitch, (size_t)P.npw * eb, (size_t)occ->nb,
                              hipMemcpyDeviceToDevice, s));
    }
    return FOCK_OK;
  }
  if (grad_occ) {
    // dE/d conj(c_i) = 1/2 f_i (V'_x phi_i): targets act as occupied (weights g), q -> -q
    const double mq[3] = {-q[0], -q[1], -q[2]};
    st = dtype == FOCK_C128 ? apply_impl<double>(cell, P, mq, pr.q_zero, tgt, occ, w, pr.L, s, grad_occ, s0, occ->w, grad_ex)
                            : apply_impl<float>(cell, P, mq, pr.q_zero, tgt, occ, w, pr.L, s, grad_occ, s0, occ->w, grad_ex);
    if (st != FOCK_OK) return st;
  }
  return FOCK_OK;
}

size_t fock_workspace_size_kmesh(const fock_cell* cell, int32_t dtype, int32_t nk, int32_t nb_max) {
  if (!cell || nk <= 0 || nb_max < 0 || (dtype != FOCK_C128 && dtype != FOCK_C64)) return 0;
  if (!grid_supported(cell->n, dtype)) return 0;
  const long long N = (long long)cell->n[0] * cell->n[1] * cell->n[2];
  const int ngroups = cell->n[1] * cell->n[2] / pencil_columns(cell->n[0], tbytes_of(dtype));
  return layout_kmesh(N, dtype == FOCK_C128 ? 16 : 8, ngroups, nk, nb_max).total;
}

fock_status fock_energy_kmesh(const fock_cell* cell, int32_t nk, const double* kpts, int32_t dtype,
                              const fock_orbs* sets, double* ex_out, void* ws, size_t ws_bytes, void* stream) {
  std::shared_ptr<Plan> plan;
  Layout L;
  fock_status st = kmesh_prepare(cell, nk, kpts, dtype, sets, ws, ws_bytes, &plan, &L);
  if (st != FOCK_OK) return st;
  if (!ex_out) return fail(FOCK_E_ARG, "ex_out is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  if (dtype == FOCK_C128) return kmesh_impl<double>(cell, *plan, nk, kpts, sets, w, L, s, ex_out, nullptr, nullptr);
  return kmesh_impl<float>(cell, *plan, nk, kpts, sets, w, L, s, ex_out, nullptr, nullptr);
}

fock_status fock_energy_kmesh_backward(const fock_cell* cell, int32_t nk, const double* kpts, int32_t dtype,
                                       const fock_orbs* sets, const double* grad_ex, void* const* grad, void* ws,
                                       size_t ws_bytes, void* stream) {
  std::shared_ptr<Plan> plan;
  Layout L;
  fock_status st = kmesh_prepare(cell, nk, kpts, dtype, sets, ws, ws_bytes, &plan, &L);
  if (st != FOCK_OK) return st;
  if (!grad_ex || !grad) return fail(FOCK_E_ARG, "grad_ex and grad must not be NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  if (dtype == FOCK_C128) return kmesh_impl<double>(cell, *plan, nk, kpts, sets, w, L, s, nullptr, grad_ex, grad);
  return kmesh_impl<float>(cell, *plan, nk, kpts, sets, w, L, s, nullptr, grad_ex, grad);
}

fock_status fock_energy_kmesh_grad(const fock_cell* cell, int32_t nk, const double* kpts, int32_t dtype,
                                   const fock_orbs* sets, double* ex_out, void* const* grad, void* ws,
                                   size_t ws_bytes, void* stream) {
  if (!ex_out || !grad) return fail(FOCK_E_ARG, "ex_out and grad must not be NULL");
  if (sets && nk > 0)
    for (int k = 0; k < nk; ++k)
      if (sets[k].nb > 0 && !grad[k]) return fail(FOCK_E_ARG, "grad[" + std::to_string(k) + "] is NULL");
  std::shared_ptr<Plan> plan;
  Layout L;
  fock_status st = kmesh_prepare(cell, nk, kpts, dtype, sets, ws, ws_bytes, &plan, &L);
  if (st != FOCK_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  if (dtype == FOCK_C128) return kmesh_impl<double>(cell, *plan, nk, kpts, sets, w, L, s, ex_out, nullptr, grad, true);
  return kmesh_impl<float>(cell, *plan, nk, kpts, sets, w, L, s, ex_out, nullptr, grad, true);
}

fock_status fock_fft3d(const int32_t n[3], int32_t dtype, int32_t sign, void* x, int32_t nb, void* stream) {
  if (!n) return fail(FOCK_E_ARG, "n is NULL");
  if (dtype != FOCK_C128 && dtype != FOCK_C64) return fail(FOCK_E_ARG, "bad dtype");
  if (sign != 1 && sign != -1) return fail(FOCK_E_ARG, "sign must be +1 or -1");
  if (nb < 0) return fail(FOCK_E_ARG, "nb < 0");
  if (nb > 0 && !x) return fail(FOCK_E_ARG, "x is NULL");
  int nn[3] = {n[0], n[1], n[2]};
  if (!grid_supported(nn, dtype)) return fail(FOCK_E_UNSUPPORTED_GRID, "no compiled transforms for grid " + grid_str(nn));
  std::shared_ptr<Plan> p;
  fock_status st = make_fft_plan(nn, dtype, &p);
  if (st != FOCK_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dtype == FOCK_C128) return Engine<double>(*p, s).transform(x, nb, sign);
  return Engine<float>(*p, s).transform(x, nb, sign);
}

size_t fock_band_workspace_size(const fock_cell* cell, int32_t dtype, int32_t nb) {
  if (!cell || nb < 0 || (dtype != FOCK_C128 && dtype != FOCK_C64)) return 0;
  if (!grid_supported(cell->n, dtype)) return 0;
  const long long N = (long long)cell->n[0] * cell->n[1] * cell->n[2];
  return band_layout(N, dtype == FOCK_C128 ? 16 : 8, nb).total;
}

fock_status fock_band_density(const fock_cell* cell, int32_t dtype, const fock_orbs* orbs, double* rho_out, void* ws,
                              size_t ws_bytes, void* stream) {
  std::shared_ptr<Plan> P;
  BandLayout L;
  fock_status st = band_prepare(cell, dtype, orbs, ws, ws_bytes, &P, &L);
  if (st != FOCK_OK) return st;
  if (!rho_out) return fail(FOCK_E_ARG, "rho_out is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  if (dtype == FOCK_C128) return band_density_impl<double>(*P, orbs, rho_out, w, L, s);
  return band_density_impl<float>(*P, orbs, rho_out, w, L, s);
}

fock_status fock_band_force(const fock_cell* cell, const double k[3], int32_t dtype, const fock_orbs* orbs,
                            const void* vloc, void* force_out, void* ws, size_t ws_bytes, void* stream) {
  if (!k) return fail(FOCK_E_ARG, "k is NULL");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(k[a])) return fail(FOCK_E_ARG, "k must be finite");
  std::shared_ptr<Plan> P;
  BandLayout L;
  fock_status st = band_prepare(cell, dtype, orbs, ws, ws_bytes, &P, &L);
  if (st != FOCK_OK) return st;
  if (orbs->nb > 0 && (!vloc || !force_out)) return fail(FOCK_E_ARG, "vloc and force_out must not be NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  if (dtype == FOCK_C128) return band_force_impl<double>(*P, k, orbs, vloc, force_out, w, L, s);
  return band_force_impl<float>(*P, k, orbs, vloc, force_out, w, L, s);
}

fock_status fock_exchange_grid(const fock_cell* cell, int32_t nq, const double* q, int32_t dtype, int32_t n_out[3]) {
  if (!cell || !n_out) return fail(FOCK_E_ARG, "cell and n_out must not be NULL");
  if (dtype != FOCK_C128 && dtype != FOCK_C64) return fail(FOCK_E_ARG, "bad dtype");
  if (cell->npw <= 0 || !cell->miller) return fail(FOCK_E_ARG, "empty G-sphere (npw <= 0 or miller NULL)");
  if (nq < 0 || (nq > 0 && !q)) return fail(FOCK_E_ARG, "need nq >= 0 and q for nq > 0");
  if (std::isnan(cell->ecut_fock)) return fail(FOCK_E_ARG, "ecut_fock is NaN");
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      if (!std::isfinite(cell->a[i][j])) return fail(FOCK_E_ARG, "lattice vectors must be finite");
  for (int j = 0; j < 3 * nq; ++j)
    if (!std::isfinite(q[j])) return fail(FOCK_E_ARG, "q must be finite");
  int need[3];
  alias_need(cell, q, nq, need);
  static const int sizes[] = {24, 48, 64, 72, 96, 128};
  long long best = -1;
  int pick[3] = {0, 0, 0};
  for (int n1 : sizes)
    for (int n2 : sizes)
      for (int n3 : sizes) {
        const int n[3] = {n1, n2, n3};
        if (n1 < need[0] || n2 < need[1] || n3 < need[2] || !grid_supported(n, dtype)) continue;
        const long long N = (long long)n1 * n2 * n3;
        if (best < 0 || N < best) {
          best = N;
          pick[0] = n1;
          pick[1] = n2;
          pick[2] = n3;
        }
      }
  if (best < 0) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "no compiled grid reaches %d x %d x %d", need[0], need[1], need[2]);
    return fail(FOCK_E_UNSUPPORTED_GRID, buf);
  }
  for (int k = 0; k < 3; ++k) n_out[k] = pick[k];
  return FOCK_OK;
}

fock_status fock_batch_plan_create(const fock_cell* cells, const fock_orbs* occ, const fock_orbs* tgt,
                                   const double (*q)[3], int32_t nsys, int32_t dtype, const char* tune_cache,
                                   void** plan) {
  if (!plan) return fail(FOCK_E_ARG, "plan is NULL");
  *plan = nullptr;
  if (nsys <= 0 || !cells || !occ) return fail(FOCK_E_ARG, "need nsys > 0, cells and occ");
  if (dtype != FOCK_C128 && dtype != FOCK_C64) return fail(FOCK_E_ARG, "bad dtype");
  auto B = std::make_unique<BatchPlanImpl>();
  B->dtype = dtype;
  B->nsys = nsys;
  fock_status st;
  for (int k = 0; k < nsys; ++k) {
    const fock_cell* c = &cells[k];
    const fock_orbs& o = occ[k];
    const fock_orbs& t = tgt ? tgt[k] : occ[k];
    const double q0[3] = {0.0, 0.0, 0.0};
    const double* qk = q ? q[k] : q0;
    if ((st = check_cell_host(c, dtype)) != FOCK_OK) return st;
    if (!grid_supported(c->n, dtype)) return fail(FOCK_E_UNSUPPORTED_GRID, "unsupported grid " + grid_str(c->n));
    if ((st = check_orbs(&o, c->npw, "occ[k]")) != FOCK_OK) return st;
    if ((st = check_orbs(&t, c->npw, "tgt[k]")) != FOCK_OK) return st;
    bool qz = true;
    if ((st = check_q(c, qk, &qz)) != FOCK_OK) return st;
    if ((st = check_alias(c, qk, 1)) != FOCK_OK) return st;
    const bool self = o.c == t.c && o.nb == t.nb && o.ld == t.ld;
    const bool cubic = c->n[0] == c->n[1] && c->n[1] == c->n[2] &&
                       (c->n[0] == 24 || c->n[0] == 48 || c->n[0] == 64 || c->n[0] == 72 || c->n[0] == 96);
    if (!(self && qz && cubic)) B->persistent_ok = false;
    B->tgt.push_back(t);
    B->q.insert(B->q.end(), qk, qk + 3);
    B->qzero.push_back(qz ? 1 : 0);
  }
  if (hipGetDevice(&B->device) != hipSuccess) return fail(FOCK_E_HIP, "no HIP device available");
  hipDeviceProp_t prop{};
  if (hipGetDeviceProperties(&prop, B->device) != hipSuccess) return fail(FOCK_E_HIP, "hipGetDeviceProperties failed");
  B->cus = prop.multiProcessorCount;
  for (int k = 0; k < nsys; ++k) {
    std::shared_ptr<Plan> P;
    if ((st = get_plan(&cells[k], dtype, &P)) != FOCK_OK) return st;
    B->plans.push_back(P);
    fock_cell c = cells[k];
    c.miller = nullptr;  // host memory of the caller: not kept
    B->cells.push_back(c);
    B->orbs.push_back(occ[k]);
  }
  const char* env_cache = std::getenv("FOCK_TUNE_CACHE");
  const std::string cache = tune_cache ? tune_cache : (env_cache ? env_cache : "");
  st = dtype == FOCK_C128 ? batch_create<double>(*B, cache) : batch_create<float>(*B, cache);
  if (st != FOCK_OK) return st;
  *plan = B.release();
  return FOCK_OK;
}

fock_status fock_batch_apply(void* plan, void* const* vx_out, double* ex_out, void* stream) {
  if (!plan) return fail(FOCK_E_ARG, "plan is NULL");
  BatchPlanImpl* B = static_cast<BatchPlanImpl*>(plan);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipGraphLaunch(B->exec, s);
  if (e != hipSuccess) return fail(FOCK_E_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
  const size_t cb = B->dtype == FOCK_C128 ? 16 : 8;
  for (int k = 0; vx_out && k < B->nsys; ++k) {
    const fock_orbs& t = B->tgt[k];
    if (!vx_out[k] || t.nb == 0) continue;
    // rows of npw values at the targets' leading dimension; entries p >= npw untouched
    e = hipMemcpy2DAsync(vx_out[k], cb * t.ld, B->outs[k], cb * t.ld, cb * B->plans[k]->npw, t.nb,
                         hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return fail(FOCK_E_HIP, std::string("batch result copy: ") + hipGetErrorString(e));
  }
  if (ex_out) {
    e = hipMemcpyAsync(ex_out, B->d_ex, sizeof(double) * B->nsys, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return fail(FOCK_E_HIP, std::string("batch energy copy: ") + hipGetErrorString(e));
  }
  return FOCK_OK;
}

fock_status fock_batch_check(void* plan) {
  if (!plan) return fail(FOCK_E_ARG, "plan is NULL");
  BatchPlanImpl* B = static_cast<BatchPlanImpl*>(plan);
  int aborted = 0;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(&aborted, B->d_abort, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(FOCK_E_HIP, std::string("batch check: ") + hipGetErrorString(e));
  if (aborted) return fail(FOCK_E_HIP, "batch scheduler aborted a dependency wait");
  return FOCK_OK;
}

fock_status fock_batch_set_wait_limit(void* plan, double ms) {
  if (!plan) return fail(FOCK_E_ARG, "plan is NULL");
  if (std::isnan(ms)) return fail(FOCK_E_ARG, "ms is NaN");
  BatchPlanImpl* B = static_cast<BatchPlanImpl*>(plan);
  (void)hipSetDevice(B->device);
  return batch_set_wait(*B, ms > 0.0 ? ms : B->wait_ms);
}

const char* fock_batch_plan_info(void* plan) {
  if (!plan) return "";
  return static_cast<BatchPlanImpl*>(plan)->info.c_str();
}

void fock_batch_plan_destroy(void* plan) { delete static_cast<BatchPlanImpl*>(plan); }

const char* fock_status_string(fock_status st) {
  switch (st) {
    case FOCK_OK: return "ok";
    case FOCK_E_ARG: return "invalid argument";
    case FOCK_E_ALIAS: return "G-sphere does not fit the grid without aliasing";
    case FOCK_E_SINGULAR_Q: return "q + G = 0 for a non-zero q";
    case FOCK_E_WORKSPACE: return "workspace too small";
    case FOCK_E_UNSUPPORTED_GRID: return "unsupported FFT grid";
    case FOCK_E_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

const char* fock_last_error(void) { return g_last_error.c_str(); }

int fock_trace_enable(int on) {
  Tracer& T = tracer();
  std::lock_guard<std::mutex> lk(T.m);
  T.on = on != 0;
  return KC_COUNT;
}

int fock_trace_read(double* ms_out, long long* count_out, int reset) {
  Tracer& T = tracer();
  std::lock_guard<std::mutex> lk(T.m);
  for (auto& r : T.recs) {
    float ms = 0.0f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      T.ms[r.k] += ms;
      T.n[r.k] += 1;
    }
    T.pool.push_back(r.a);
    T.pool.push_back(r.b);
  }
  T.recs.clear();
  for (int k = 0; k < KC_COUNT; ++k) {
    if (ms_out) ms_out[k] = T.ms[k];
    if (count_out) count_out[k] = T.n[k];
    if (reset) {
      T.ms[k] = 0.0;
      T.n[k] = 0;
    }
  }
  return KC_COUNT;
}

const char* fock_trace_name(int k) { return (k >= 0 && k < KC_COUNT) ? kClassNames[k] : ""; }

void fock_release_plans(void) {
  std::lock_guard<std::mutex> lk(g_mutex);
  g_plans.clear();
  g_fft_plans.clear();
}

}  // extern "C"
