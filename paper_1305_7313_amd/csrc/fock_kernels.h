// Device kernels of the exact-exchange band-pair path (section 4 of Varini et
// al., "Enhancement of DFT-calculations at Petascale"):
//
//   a1  orbitals to real space:  scatter the sphere, backward 3-D FFT
//   P1  pair density conj(phi_i) psi_j  +  forward FFT over the plane axes
//   P2  forward FFT along axis 1, Coulomb kernel K(q+G) (+ FP64 energy
//       partials), backward FFT along axis 1
//   P3  backward FFT over the plane axes, multiply by f_i phi_i, accumulate
//       over the occupied tile into (V_x psi)_j in real space
//   a7  per target: forward 3-D FFT, gather the sphere, scale
//
// The FFT box is C order [n1][n2][n3]; a "plane" is one i1 slice (n2*n3
// contiguous values), a "pencil" runs along i1 with stride n2*n3.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "fft_engine.h"

namespace fockx {

constexpr double kFourPi = 12.566370614359172953850573533118011536788677597500;

enum PlaneMode : int {
  PLANE_PAIR_FWD = 0,  // P1
  PLANE_INV_MAC = 1,   // P3
  PLANE_FWD = 2,       // in place, forward (a7)
  PLANE_INV = 3,       // in place, backward (a1)
  PLANE_INV_MAC_MIR = 4,  // P3, mirrored half of the pair-symmetric schedule
  PLANE_DENS = 5,      // band loop: backward plane FFT, accumulate w |psi|^2
  PLANE_VMUL = 6,      // band loop, in place: backward plane FFT, x V(r), forward plane FFT
  // Gamma point, real orbitals packed two per complex array (P_q = psi_2q + i psi_2q+1)
  PLANE_PAIR_FWD_G = 7,    // P1: phi_i(r) P_q(r), forward plane FFT
  PLANE_INV_MAC_G = 8,     // P3 into the packed targets' accumulators
  PLANE_INV_MAC_MIR_G = 9, // P3 mirror into the occupied orbitals' accumulator components
};
enum PencilMode : int {
  PENCIL_FKI = 0,  // P2: forward, kernel, backward (+ optional energy partials)
  PENCIL_FE = 1,   // forward + energy partials only
  PENCIL_FWD = 2,  // in place, forward (a7)
  PENCIL_INV = 3,  // in place, backward (a1)
};

// What the kernel needs to evaluate K(q+G) at G = m1 b1 + m2 b2 + m3 b3.
struct KernelParams {
  double b[3][3];      // reciprocal lattice vectors (rows), bohr^-1
  double q[3];         // bohr^-1
  double ecut;         // cutoff on |q+G|^2; <= 0: none
  const double* k0;    // device scalar: K at q+G = 0 (only used when q_zero)
  int q_zero;
};

struct PlaneArgs {
  void* x;             // in-place modes: [nb][N]
  const void* a;       // occupied orbitals in real space [*][N]
  const void* bsrc;    // target orbitals in real space [*][N]
  void* w;             // pair buffer [ti*tj][N], slot = ii*tj + jj
  void* acc;           // accumulators [tj][N]
  const double* f;     // occupied weights, absolute index
  const void* tw2;     // twiddle table, length n2
  const void* tw3;     // twiddle table, length n3
  long long N;
  int i0, j0, ti, tj;  // tile origin and extent
  int n1, nb;
  double fscale;       // constant factor on f in P3
  int store_v;         // P3: also write the real-space v back into the pair buffer
  // band loops (PLANE_DENS, PLANE_VMUL): workgroup (i1, group g) takes the
  // bands g, g + ngrp, ... < nb of x
  int ngrp;
  double* part;        // PLANE_DENS: FP64 partial densities [ngrp][N]
  int accumulate;      // PLANE_DENS: add to part (else overwrite)
  const void* vloc;    // PLANE_VMUL: real potential V(r) [N], path precision
  int nreal;           // Gamma modes: number of real orbitals (packed arrays hold ceil(nreal / 2))
  int tri;             // diagonal tile of a self-application (i0 == j0, ti == tj): only the
                       // pairs ii <= jj, pair buffer slot tri_slot(ii, jj)
  const signed char* live;  // pair-buffer planes: per column i3 the last live row
                            // (live_row); null: every entry is live
};

// Row i2 of plane column with bound h (|m2| <= h, h < 0: empty column) holds
// pair-density data; entries outside are zero and are neither stored nor read.
template <int N2> __device__ __forceinline__ bool live_row(int i2, int h) { return i2 <= h || i2 >= N2 - h; }

// Slot of pair (ii, jj), ii <= jj, in the pair buffer of a diagonal tile.
__host__ __device__ constexpr int tri_slot(int ii, int jj) { return jj * (jj + 1) / 2 + ii; }

// Gamma diagonal tile (real occupied i0 = 2 j0): packed target jj needs the
// occupied ii < gtri_count(ti, jj) (i <= 2q + 1; the rest have zero weights),
// stored from slot gtri_prefix(ti, jj).
__host__ __device__ constexpr int gtri_count(int ti, int jj) { return ti < 2 * jj + 2 ? ti : 2 * jj + 2; }
__host__ __device__ constexpr int gtri_prefix(int ti, int jj) {
  int s = 0;
  for (int j = 0; j < jj; ++j) s += gtri_count(ti, j);
  return s;
}

// Both maps enumerate their pairs exactly once, in slots 0 .. count - 1.
constexpr bool compact_slots_ok() {
  for (int t = 1; t <= 16; ++t) {
    bool seen[136] = {};
    for (int jj = 0; jj < t; ++jj)
      for (int ii = 0; ii <= jj; ++ii) {
        const int s = tri_slot(ii, jj);
        if (s < 0 || s >= tri_slot(0, t) || seen[s]) return false;
        seen[s] = true;
      }
  }
  for (int ti = 1; ti <= 16; ++ti)
    for (int tj = 1; tj <= 8; ++tj) {
      bool seen[128] = {};
      int n = 0;
      for (int jj = 0; jj < tj; ++jj)
        for (int ii = 0; ii < ti; ++ii) {
          if (ii > 2 * jj + 1) continue;  // i > 2q + 1: all weights zero
          const int s = gtri_prefix(ti, jj) + ii;
          if (ii >= gtri_count(ti, jj) || s >= gtri_prefix(ti, tj) || seen[s]) return false;
          seen[s] = true;
          ++n;
        }
      if (n != gtri_prefix(ti, tj)) return false;
    }
  return tri_slot(0, 16) == 136 && gtri_prefix(16, 8) == 72;
}
static_assert(compact_slots_ok(), "compact diagonal-tile slot maps");

struct PencilArgs {
  const signed char* live;  // pair buffers: last live row per plane column (see PlaneArgs), or null
  void* x;             // [npairs or nb][N]
  double* epart;       // PENCIL_FE: energy partials [ngroups][npairs] (group-major)
  const void* tw1;     // twiddle table, length n1
  KernelParams kp;
  long long N;
  int n2, n3, count;   // count = pairs or orbitals
  int skip_dead;       // PENCIL_FKI with live: 1 leaves the lines of wholly dead columns
                       // unwritten (every reader of this buffer masks them); 0 writes the zeros
};

// Hardware dispatches workgroup w to XCD (w mod 8).  Renumber so that
// consecutive logical blocks run on the same XCD and share its L2.
__device__ __forceinline__ int xcd_logical(int w, int G) {
  const int x = w & 7, slot = w >> 3;
  const int per = G >> 3, extra = G & 7;
  return x * per + (x < extra ? x : extra) + slot;
}

template <typename T>
__device__ __forceinline__ void load_table(cx<T>* dst, const void* src, int n) {
  const cx<T>* s = reinterpret_cast<const cx<T>*>(src);
  for (int k = threadIdx.x; k < n; k += blockDim.x) dst[k] = s[k];
}

__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int k = 0; k < nw; ++k) s += red[k];
  }
  return s;
}

__device__ __forceinline__ int signed_index(int i, int n) { return i < (n >> 1) ? i : i - n; }

// ---------------------------------------------------------------------------
// Plane kernel: 2-D FFT over (i2, i3) of one i1 plane.
// ---------------------------------------------------------------------------

// Plane body: W threads, SPLIT selects the 8-byte (two-round) LDS exchange.
// Per-exchange LDS layouts (fft_engine.h, Tile) on every plane but the FP32
// 96 x 96 one, which keeps the compact tile: the larger one costs it the
// second resident workgroup per CU (+15%).
template <typename T, int N3> constexpr bool plane_tile_pad() { return !(sizeof(T) == 4 && N3 == 96); }

template <typename T, int N2, int N3, int W, bool SPLIT> struct PlaneGeom {
  static constexpr int PLANE = N2 * N3;
  static constexpr int XBYTES =
      plane_slots<N3, plane_tile_pad<T, N3>()>(N2) * (SPLIT ? (int)sizeof(T) : 2 * (int)sizeof(T));
  // transforms along i3, one per row.  On the compact (unpadded) tile the
  // rows take the larger radix first: a forward first row pass then writes
  // column R1 i + r from lane i (for 96: 12 i + r), which with the odd row
  // stride gives each of 32 lanes served together its own pair of banks.
  using Rw = std::conditional_t<plane_tile_pad<T, N3>(), Axis<N3, N2, true, W>,
                                Axis<N3, N2, true, W, Factor<N3>::R1, Factor<N3>::R0>>;
  using Cl = Axis<N2, N3, false, W>;  // transforms along i2, one per column
  static constexpr int NV = Rw::NV > Cl::NV ? Rw::NV : Cl::NV;
};

template <typename T, int N2, int N3, int W, bool SPLIT, int MODE>
__device__ __forceinline__ void plane_body(const PlaneArgs& A, int lid, unsigned char* smem, const cx<T>* tw2,
                                           const cx<T>* tw3) {
  using Cfg = PlaneGeom<T, N2, N3, W, SPLIT>;
  constexpr bool PAD = plane_tile_pad<T, N3>();
  // On the compact (unpadded) tile, the row pass that touches only LDS walks
  // the rows with its lanes: the forward direction's second row pass, the
  // backward direction's first.  Its exchanges then spread the lanes of a
  // wave over 32 rows at the odd stride COLS + 1, one bank pair each,
  // instead of over strided columns of a few rows.  The V-multiply mode,
  // whose row passes also meet V(r) in HBM, keeps the default order.
  constexpr bool fwd_dir = MODE == PLANE_PAIR_FWD || MODE == PLANE_PAIR_FWD_G || MODE == PLANE_FWD;
  constexpr bool rows_lb = !PAD && MODE != PLANE_VMUL;
  using R0 = std::conditional_t<rows_lb && !fwd_dir, typename Cfg::Rw::P0b, typename Cfg::Rw::P0>;
  using R1 = std::conditional_t<rows_lb && fwd_dir, typename Cfg::Rw::P1b, typename Cfg::Rw::P1>;
  using C0 = typename Cfg::Cl::P0;
  using C1 = typename Cfg::Cl::P1;
  constexpr int PLANE = Cfg::PLANE;
  const int t = threadIdx.x;
  const long long N = A.N;
  cx<T> v[Cfg::NV];

  if constexpr (MODE == PLANE_PAIR_FWD || MODE == PLANE_PAIR_FWD_G) {
    // workgroup (i1, slot): slot = ii * tj + jj, or on a diagonal tile
    // tri_slot(ii, jj) (gtri_prefix(ti, jj) + ii in the Gamma modes)
    constexpr bool gam = MODE == PLANE_PAIR_FWD_G;
    const int tt = A.tri ? (gam ? gtri_prefix(A.ti, A.tj) : A.ti * (A.ti + 1) / 2) : A.ti * A.tj;
    const int i1 = lid / tt, rem = lid - i1 * tt;
    int ii, jj;
    if (A.tri && gam) {
      jj = 0;
      int base = 0;
      while (rem >= base + gtri_count(A.ti, jj)) base += gtri_count(A.ti, jj++);
      ii = rem - base;
    } else if (A.tri) {
      jj = 0;
      while (tri_slot(0, jj + 1) <= rem) ++jj;
      ii = rem - tri_slot(0, jj);
    } else {
      ii = rem / A.tj;
      jj = rem - ii * A.tj;
    }
    const cx<T>* pb = reinterpret_cast<const cx<T>*>(A.bsrc) + (long long)(A.j0 + jj) * N + (long long)i1 * PLANE;
    if constexpr (MODE == PLANE_PAIR_FWD) {
      const cx<T>* pa = reinterpret_cast<const cx<T>*>(A.a) + (long long)(A.i0 + ii) * N + (long long)i1 * PLANE;
      for_inputs<R0>(t, [&](int e, int row, int col) {
        const int p = row * N3 + col;
        v[e] = cmulc<T>(pa[p], pb[p]);
      });
    } else {
      // real phi_i is one component of the packed occupied array
      const int i = A.i0 + ii;
      const cx<T>* pa = reinterpret_cast<const cx<T>*>(A.a) + (long long)(i >> 1) * N + (long long)i1 * PLANE;
      const bool hi = i & 1;
      for_inputs<R0>(t, [&](int e, int row, int col) {
        const int p = row * N3 + col;
        const cx<T> a = pa[p];
        v[e] = cscale<T>(pb[p], hi ? a.y : a.x);
      });
    }
    pass_compute<R0, -1, T>(v, tw3, t);
    exchange<R0, R1, N3, SPLIT, T, PAD>(v, smem, t);
    pass_compute<R1, -1, T>(v, tw3, t);
    exchange<R1, C0, N3, SPLIT, T, PAD>(v, smem, t);
    pass_compute<C0, -1, T>(v, tw2, t);
    exchange<C0, C1, N3, SPLIT, T, PAD>(v, smem, t);
    pass_compute<C1, -1, T>(v, tw2, t);
    cx<T>* pw = reinterpret_cast<cx<T>*>(A.w) + (long long)rem * N + (long long)i1 * PLANE;
    const int hc = A.live ? A.live[t % N3] : N2;  // a column pass: column t % N3 for every value
    // Dead entries are not stored.  On the 128-wide rows a 128-byte line
    // with a live entry is written whole (the dead entries' values are never
    // read), since a partly written line costs the memory a read-modify-write;
    // measured there: P1 -7% (FP64) and -1.4% (FP32), where the 96-wide FP32
    // and 64-wide FP64 rows lose 3% and 9% to the extra bytes and keep their
    // per-entry stores.  The LINE lanes of an aligned lane group hold one
    // line of one row (consecutive columns from a multiple of N3).
    constexpr int LINE = 128 / (int)sizeof(cx<T>);
    for_outputs<C1>(t, [&](int e, int row, int col) {
      bool st = live_row<N2>(row, hc);
      if constexpr (N3 == 128) {
        if (A.live) {
          const unsigned long long m = __ballot(st);
          st = ((m >> ((t & 63) & ~(LINE - 1))) & ((1ull << LINE) - 1)) != 0;
        }
      }
      if (st) store_stream<T>(&pw[row * N3 + col], v[e]);
    });
  } else if constexpr (MODE == PLANE_INV_MAC || MODE == PLANE_INV_MAC_MIR) {
    // PLANE_INV_MAC: block (jj, i1), loop over ii, acc_j += f_i phi_i v_ij.
    // PLANE_INV_MAC_MIR (one orbital block at q = 0): block (ii, i1), loop over
    // jj, acc_i += f_j phi_j conj(v_ij), since v_ji = conj(v_ij).
    // On a diagonal tile (tri) the forward pass takes ii <= jj and the mirror
    // ii < jj, so each unordered pair reaches each accumulator once.
    constexpr bool mir = MODE == PLANE_INV_MAC_MIR;
    const int nblk = mir ? A.ti : A.tj, nloop = mir ? A.tj : A.ti;
    const int i1 = lid / nblk, bi = lid - (lid / nblk) * nblk;
    const int o0 = mir ? A.j0 : A.i0;
    const cx<T>* src = reinterpret_cast<const cx<T>*>(mir ? A.bsrc : A.a);
    const int k0 = A.tri && mir ? bi + 1 : 0, k1 = A.tri && !mir ? bi + 1 : nloop;
    // every entry is read here: skipping the dead columns (zeros) measured
    // slower in these register-heavy passes than reading them
    cx<T> s[R1::NV];
#pragma unroll
    for (int e = 0; e < R1::NV; ++e) s[e] = mk<T>(T(0), T(0));
    for (int k = k0; k < k1; ++k) {
      const int slot = A.tri ? (mir ? tri_slot(bi, k) : tri_slot(k, bi)) : (mir ? bi * A.tj + k : k * A.tj + bi);
      const cx<T>* pw = reinterpret_cast<const cx<T>*>(A.w) + (long long)slot * N + (long long)i1 * PLANE;
      for_inputs<C0>(t, [&](int e, int row, int col) { v[e] = load_stream<T>(&pw[row * N3 + col]); });
      pass_compute<C0, +1, T>(v, tw2, t);
      exchange<C0, C1, N3, SPLIT, T, PAD>(v, smem, t);
      pass_compute<C1, +1, T>(v, tw2, t);
      exchange<C1, R0, N3, SPLIT, T, PAD>(v, smem, t);
      pass_compute<R0, +1, T>(v, tw3, t);
      exchange<R0, R1, N3, SPLIT, T, PAD>(v, smem, t);
      pass_compute<R1, +1, T>(v, tw3, t);
      const T fk = T(A.f[o0 + k] * A.fscale);
      const cx<T>* pa = src + (long long)(o0 + k) * N + (long long)i1 * PLANE;
      if (!mir && A.store_v) {
        cx<T>* pv = const_cast<cx<T>*>(pw);
        for_outputs<R1>(t, [&](int e, int row, int col) { pv[row * N3 + col] = v[e]; });
      }
      if constexpr (mir) {
        for_outputs<R1>(t, [&](int e, int row, int col) {
          const cx<T> pr = cmulc<T>(v[e], pa[row * N3 + col]);  // conj(v) phi
          s[e] = mk<T>(s[e].x + fk * pr.x, s[e].y + fk * pr.y);
        });
      } else {
        for_outputs<R1>(t, [&](int e, int row, int col) {
          const cx<T> pr = cmul<T>(pa[row * N3 + col], v[e]);
          s[e] = mk<T>(s[e].x + fk * pr.x, s[e].y + fk * pr.y);
        });
      }
    }
    cx<T>* pc = reinterpret_cast<cx<T>*>(A.acc) + (long long)bi * N + (long long)i1 * PLANE;
    for_outputs<R1>(t, [&](int e, int row, int col) {
      const int p = row * N3 + col;
      pc[p] = cadd<T>(pc[p], s[e]);
    });
  } else if constexpr (MODE == PLANE_INV_MAC_G || MODE == PLANE_INV_MAC_MIR_G) {
    // Gamma tiles: real occupied i = i0 + ii, packed targets q = j0 + jj with
    // v = v_{i,2q} + i v_{i,2q+1}.  Each unordered pair counts once per
    // accumulator: a pair (i, j) adds f_i phi_i v_ij to acc_j when i <= j and
    // f_j phi_j v_ij to acc_i when i < j (the weights below vanish otherwise,
    // which only happens on the diagonal tiles).
    // PLANE_INV_MAC_G: block (jj, i1), loop over ii, into packed acc_q.
    // PLANE_INV_MAC_MIR_G: block (ii, i1), loop over jj, into component
    // (i & 1) of packed acc_{i/2} (acc points at the tile's first pair).
    // On a diagonal tile (tri) only the stored pairs ii < gtri_count(ti, jj) are visited.
    constexpr bool mir = MODE == PLANE_INV_MAC_MIR_G;
    const int nblk = mir ? A.ti : A.tj, nloop = mir ? A.tj : A.ti;
    const int i1 = lid / nblk, bi = lid - (lid / nblk) * nblk;
    int k0 = 0, k1 = nloop;
    if (A.tri) {
      if (mir) k0 = bi / 2;  // first jj with bi < 2 jj + 2
      else k1 = gtri_count(A.ti, bi);
    }
    const int hc = A.live ? A.live[t % N3] : N2;  // entries outside are zero: not read
    cx<T> s[R1::NV];
#pragma unroll
    for (int e = 0; e < R1::NV; ++e) s[e] = mk<T>(T(0), T(0));
    for (int k = k0; k < k1; ++k) {
      const int ii = mir ? bi : k, jj = mir ? k : bi;
      const int i = A.i0 + ii, q = A.j0 + jj;
      const int j0r = 2 * q, j1r = 2 * q + 1;
      const int slot = A.tri ? gtri_prefix(A.ti, jj) + ii : ii * A.tj + jj;
      const cx<T>* pw = reinterpret_cast<const cx<T>*>(A.w) + (long long)slot * N + (long long)i1 * PLANE;
      for_inputs<C0>(t, [&](int e, int row, int col) {
        v[e] = live_row<N2>(row, hc) ? load_stream<T>(&pw[row * N3 + col]) : mk<T>(T(0), T(0));
      });
      pass_compute<C0, +1, T>(v, tw2, t);
      exchange<C0, C1, N3, SPLIT, T, PAD>(v, smem, t);
      pass_compute<C1, +1, T>(v, tw2, t);
      exchange<C1, R0, N3, SPLIT, T, PAD>(v, smem, t);
      pass_compute<R0, +1, T>(v, tw3, t);
      exchange<R0, R1, N3, SPLIT, T, PAD>(v, smem, t);
      pass_compute<R1, +1, T>(v, tw3, t);
      if constexpr (mir) {
        const T m0 = i < j0r ? T(A.f[j0r] * A.fscale) : T(0);
        const T m1 = (i < j1r && j1r < A.nreal) ? T(A.f[j1r] * A.fscale) : T(0);
        const cx<T>* pq = reinterpret_cast<const cx<T>*>(A.bsrc) + (long long)q * N + (long long)i1 * PLANE;
        for_outputs<R1>(t, [&](int e, int row, int col) {
          const cx<T> pp = pq[row * N3 + col];
          s[e].x += m0 * pp.x * v[e].x + m1 * pp.y * v[e].y;
        });
      } else {
        const T w0 = i <= j0r ? T(A.f[i] * A.fscale) : T(0);
        const T w1 = (i <= j1r && j1r < A.nreal) ? T(A.f[i] * A.fscale) : T(0);
        const cx<T>* pa = reinterpret_cast<const cx<T>*>(A.a) + (long long)(i >> 1) * N + (long long)i1 * PLANE;
        const bool hi = i & 1;
        for_outputs<R1>(t, [&](int e, int row, int col) {
          const cx<T> a = pa[row * N3 + col];
          const T ph = hi ? a.y : a.x;
          s[e] = mk<T>(s[e].x + w0 * ph * v[e].x, s[e].y + w1 * ph * v[e].y);
        });
      }
    }
    if constexpr (mir) {
      T* pc = reinterpret_cast<T*>(reinterpret_cast<cx<T>*>(A.acc) + (long long)(bi >> 1) * N + (long long)i1 * PLANE) +
              (bi & 1);
      for_outputs<R1>(t, [&](int e, int row, int col) {
        const int p = 2 * (row * N3 + col);
        pc[p] += s[e].x;
      });
    } else {
      cx<T>* pc = reinterpret_cast<cx<T>*>(A.acc) + (long long)bi * N + (long long)i1 * PLANE;
      for_outputs<R1>(t, [&](int e, int row, int col) {
        const int p = row * N3 + col;
        pc[p] = cadd<T>(pc[p], s[e]);
      });
    }
  } else if constexpr (MODE == PLANE_FWD) {
    const int ob = lid / A.n1, i1 = lid - (lid / A.n1) * A.n1;
    cx<T>* px = reinterpret_cast<cx<T>*>(A.x) + (long long)ob * N + (long long)i1 * PLANE;
    for_inputs<R0>(t, [&](int e, int row, int col) { v[e] = px[row * N3 + col]; });
    pass_compute<R0, -1, T>(v, tw3, t);
    exchange<R0, R1, N3, SPLIT, T, PAD>(v, smem, t);
    pass_compute<R1, -1, T>(v, tw3, t);
    exchange<R1, C0, N3, SPLIT, T, PAD>(v, smem, t);
    pass_compute<C0, -1, T>(v, tw2, t);
    exchange<C0, C1, N3, SPLIT, T, PAD>(v, smem, t);
    pass_compute<C1, -1, T>(v, tw2, t);
    for_outputs<C1>(t, [&](int e, int row, int col) { px[row * N3 + col] = v[e]; });
  } else if constexpr (MODE == PLANE_DENS) {
    // sum over this group's bands of f_b * fscale * |psi_b(r)|^2 on plane i1
    const int G = A.ngrp;
    const int i1 = lid / G, g = lid - (lid / G) * G;
    T acc[R1::NV];
#pragma unroll
    for (int e = 0; e < R1::NV; ++e) acc[e] = T(0);
    for (int b = g; b < A.nb; b += G) {
      const cx<T>* px = reinterpret_cast<const cx<T>*>(A.x) + (long long)b * N + (long long)i1 * PLANE;
      for_inputs<C0>(t, [&](int e, int row, int col) { v[e] = px[row * N3 + col]; });
      pass_compute<C0, +1, T>(v, tw2, t);
      exchange<C0, C1, N3, SPLIT, T, PAD>(v, smem, t);
      pass_compute<C1, +1, T>(v, tw2, t);
      exchange<C1, R0, N3, SPLIT, T, PAD>(v, smem, t);
      pass_compute<R0, +1, T>(v, tw3, t);
      exchange<R0, R1, N3, SPLIT, T, PAD>(v, smem, t);
      pass_compute<R1, +1, T>(v, tw3, t);
      const T wb = T(A.f[A.i0 + b] * A.fscale);
      for_outputs<R1>(t, [&](int e, int row, int col) { acc[e] += wb * (v[e].x * v[e].x + v[e].y * v[e].y); });
    }
    double* pp = A.part + (long long)g * N + (long long)i1 * PLANE;
    for_outputs<R1>(t, [&](int e, int row, int col) {
      const int p = row * N3 + col;
      pp[p] = (A.accumulate ? pp[p] : 0.0) + double(acc[e]);
    });
  } else if constexpr (MODE == PLANE_VMUL) {
    // psi_b(i1, r2, r3) = backward plane FFT; times V(r); forward plane FFT
    // back into place.  V's plane stays in registers for the group's bands.
    const int G = A.ngrp;
    const int i1 = lid / G, g = lid - (lid / G) * G;
    const T* pv = reinterpret_cast<const T*>(A.vloc) + (long long)i1 * PLANE;
    T vr[R1::NV];
    for_outputs<R1>(t, [&](int e, int row, int col) { vr[e] = pv[row * N3 + col]; });
    for (int b = g; b < A.nb; b += G) {
      cx<T>* px = reinterpret_cast<cx<T>*>(A.x) + (long long)b * N + (long long)i1 * PLANE;
      for_inputs<C0>(t, [&](int e, int row, int col) { v[e] = px[row * N3 + col]; });
      pass_compute<C0, +1, T>(v, tw2, t);
      exchange<C0, C1, N3, SPLIT, T, PAD>(v, smem, t);
      pass_compute<C1, +1, T>(v, tw2, t);
      exchange<C1, R0, N3, SPLIT, T, PAD>(v, smem, t);
      pass_compute<R0, +1, T>(v, tw3, t);
      exchange<R0, R1, N3, SPLIT, T, PAD>(v, smem, t);
      pass_compute<R1, +1, T>(v, tw3, t);
      for_outputs<R1>(t, [&](int e, int row, int col) { v[e] = cscale<T>(v[e], vr[e]); });
      exchange<R1, R0, N3, SPLIT, T, PAD>(v, smem, t);
      pass_compute<R0, -1, T>(v, tw3, t);
      exchange<R0, R1, N3, SPLIT, T, PAD>(v, smem, t);
      pass_compute<R1, -1, T>(v, tw3, t);
      exchange<R1, C0, N3, SPLIT, T, PAD>(v, smem, t);
      pass_compute<C0, -1, T>(v, tw2, t);
      exchange<C0, C1, N3, SPLIT, T, PAD>(v, smem, t);
      pass_compute<C1, -1, T>(v, tw2, t);
      for_outputs<C1>(t, [&](int e, int row, int col) { px[row * N3 + col] = v[e]; });
    }
  } else {  // PLANE_INV
    const int ob = lid / A.n1, i1 = lid - (lid / A.n1) * A.n1;
    cx<T>* px = reinterpret_cast<cx<T>*>(A.x) + (long long)ob * N + (long long)i1 * PLANE;
    const int hc = A.live ? A.live[t % N3] : N2;  // pair buffers: entries outside are zero
    for_inputs<C0>(t, [&](int e, int row, int col) {
      v[e] = live_row<N2>(row, hc) ? px[row * N3 + col] : mk<T>(T(0), T(0));
    });
    pass_compute<C0, +1, T>(v, tw2, t);
    exchange<C0, C1, N3, SPLIT, T, PAD>(v, smem, t);
    pass_compute<C1, +1, T>(v, tw2, t);
    exchange<C1, R0, N3, SPLIT, T, PAD>(v, smem, t);
    pass_compute<R0, +1, T>(v, tw3, t);
    exchange<R0, R1, N3, SPLIT, T, PAD>(v, smem, t);
    pass_compute<R1, +1, T>(v, tw3, t);
    for_outputs<R1>(t, [&](int e, int row, int col) { px[row * N3 + col] = v[e]; });
  }
}

// Default block shape per precision, plane and mode (measured on MI355X with
// a sweep of every valid block size, LDS exchange width and occupancy hint
// per plane kernel on 16 x 16 pair tiles; the fastest variant is kept).
struct PlaneTune {
  int w;
  bool split;
  int minb;  // the launch bound's minimum waves per SIMD
};
constexpr PlaneTune plane_tune(int tbytes, int n2, int n3, int mode) {
  const bool p1 = mode == PLANE_PAIR_FWD || mode == PLANE_PAIR_FWD_G, inv = mode == PLANE_INV,
             pair = p1 || inv,
             fwdmac = mode == PLANE_INV_MAC || mode == PLANE_INV_MAC_G,
             mirror = mode == PLANE_INV_MAC_MIR || mode == PLANE_INV_MAC_MIR_G,
             mac = fwdmac || mirror || mode == PLANE_DENS;
  // band loops hold an accumulator or V(r) in registers beside the plane
  const bool band = mode == PLANE_DENS || mode == PLANE_VMUL;
  if (tbytes == 8) {  // FP64
    if (band && n2 == 96 && n3 == 128) return PlaneTune{768, true, 1};
    if (n2 == 64 && n3 == 64) {
      if (p1) return PlaneTune{512, true, 1};
      if (inv) return PlaneTune{512, true, 2};
      if (mirror) return PlaneTune{512, false, 2};
      return mac ? PlaneTune{256, false, 2} : PlaneTune{256, true, 1};
    }
    // P1 at 512 threads: the only width at which its 24 values per thread fit
    // without spilling (at 768 the register cap of a 12-wave workgroup spills
    // 58 registers, and the scratch traffic doubles its HBM bytes)
    if (n2 == 96 && n3 == 128) return p1 ? PlaneTune{512, true, 1} : inv ? PlaneTune{512, true, 2} : PlaneTune{1024, true, 1};
    if (n2 == 96 && n3 == 96) return PlaneTune{768, true, 1};
    if (n2 == 72 && n3 == 72) return pair ? PlaneTune{720, true, 1} : PlaneTune{576, true, 1};
    if (n2 == 48 && n3 == 64) return PlaneTune{256, false, 1};
    if (n2 == 48 && n3 == 48) return p1 ? PlaneTune{192, true, 1} : fwdmac ? PlaneTune{384, false, 2} : PlaneTune{384, false, 1};
    return PlaneTune{192, false, 1};
  }
  if (n2 == 96 && n3 == 128) {
    if (p1) return PlaneTune{512, true, 1};
    if (inv) return PlaneTune{512, true, 1};
    return mode == PLANE_INV_MAC ? PlaneTune{512, false, 1} : PlaneTune{1024, false, 1};
  }
  if (n2 == 96 && n3 == 96) return mac ? PlaneTune{384, false, 1} : inv ? PlaneTune{768, true, 1} : PlaneTune{768, false, 1};
  if (n2 == 72 && n3 == 72) {
    // P1 and the in-place inverse at 504 threads (8 waves), re-timed on the
    // padded exchange layouts: three planes per CU in flight where two
    // workgroups of 720 threads (12 waves) fit (16-system batch 1086 -> 1071
    // ms, 72^3 k-mesh 8723 -> 8246 ms)
    if (p1) return PlaneTune{504, false, 1};
    if (fwdmac || mirror) return PlaneTune{720, false, 1};
    return inv ? PlaneTune{504, true, 1} : PlaneTune{576, false, 1};
  }
  if (n2 == 64 && n3 == 64) return p1 ? PlaneTune{256, true, 1} : PlaneTune{512, false, 1};
  if (n2 == 48 && n3 == 64) return PlaneTune{256, false, 1};
  if (n2 == 48 && n3 == 48) return p1 ? PlaneTune{192, false, 2} : PlaneTune{384, false, 1};
  return PlaneTune{192, false, 1};
}

template <typename T, int N2, int N3, int MODE> struct PlaneCfg {
  static constexpr PlaneTune P = plane_tune(sizeof(T), N2, N3, MODE);
  static constexpr int W = P.w;
  static constexpr bool SPLIT = P.split;
  static constexpr int MINB = P.minb;
};

template <typename T, int N2, int N3, int W, bool SPLIT, int MODE, int MINB>
__global__ __launch_bounds__(W, MINB) void plane_kernel(PlaneArgs A) {
  using G = PlaneGeom<T, N2, N3, W, SPLIT>;
  __shared__ __align__(16) unsigned char smem[G::XBYTES];
  __shared__ cx<T> tw2[N2];
  __shared__ cx<T> tw3[N3];
  load_table<T>(tw2, A.tw2, N2);
  load_table<T>(tw3, A.tw3, N3);
  __syncthreads();
  plane_body<T, N2, N3, W, SPLIT, MODE>(A, xcd_logical(blockIdx.x, gridDim.x), smem, tw2, tw3);
}

// ---------------------------------------------------------------------------
// Pencil kernel: 1-D FFT along i1 for CB consecutive plane positions.
// ---------------------------------------------------------------------------
// cb pencils per workgroup (the host sizes grids and energy partials with
// it, so it depends on the length and precision only), w threads; split: 1/0
// forces the two-round FP64 exchange on or off, -1 takes it when the tile
// exceeds 64 KB; minb: the launch bound's minimum waves per SIMD (registers
// per thread are capped at 512 / minb).
struct PencilTune {
  int cb, w, split, minb;
};
constexpr PencilTune pencil_tune(int tbytes, int n1, int mode = -1) {
  if (n1 == 24) return PencilTune{64, 128, -1, 1};
  // FP32 P2 on 48- and 64-point pencils: 512 threads (re-timed on a full
  // 16 x 16 tile: 48: 88 -> 81 us, 64: 191 -> 180 us)
  if (n1 == 48) return tbytes == 4 && mode == PENCIL_FKI ? PencilTune{64, 512, -1, 1} : PencilTune{64, 128, -1, 1};
  if (n1 == 64) {
    // FP64 P2: 512 threads on an unsplit 66.5 KB tile, two per CU (-3.5%)
    if (tbytes == 8 && mode == PENCIL_FKI) return PencilTune{64, 512, 0, 2};
    if (mode == PENCIL_FKI) return PencilTune{64, 512, -1, 1};
    return PencilTune{64, 256, -1, 1};
  }
  if (n1 == 72) return tbytes == 4 ? PencilTune{32, 128, -1, 1} : PencilTune{32, 256, -1, 1};
  if (n1 == 96) return tbytes == 4 ? PencilTune{64, 512, -1, 1} : PencilTune{32, 256, -1, 1};
  return PencilTune{32, 256, -1, 1};
}

template <typename T, int N1, int CB, int W, bool SPLIT> struct PencilGeom {
  static constexpr int XBYTES = Tile<CB>::slots(N1) * (SPLIT ? (int)sizeof(T) : 2 * (int)sizeof(T));
  using Ax = Axis<N1, CB, false, W>;
  static constexpr int NV = Ax::NV;
};

template <typename T, int N1, int CB, int W, bool SPLIT, int MODE>
__device__ __forceinline__ void pencil_body(const PencilArgs& A, int lid, unsigned char* smem, const cx<T>* tw1,
                                            double* red) {
  using Cfg = PencilGeom<T, N1, CB, W, SPLIT>;
  using P0 = typename Cfg::Ax::P0;
  using P1 = typename Cfg::Ax::P1;
  const int t = threadIdx.x;
  const int plane = A.n2 * A.n3;
  const int ngroups = plane / CB;
  const int pr = lid / ngroups, g = lid - (lid / ngroups) * ngroups;
  const int c0 = g * CB;
  cx<T>* base = reinterpret_cast<cx<T>*>(A.x) + (long long)pr * A.N + c0;
  cx<T> v[Cfg::NV];

  // (row, col) of the tile = (i1, column c0 + col).  A column pass: every
  // value of this thread is in column c0 + t % CB.  In pair buffers (live
  // set) P1 has not stored the dead columns: those pencils are not read and
  // transform as zero.  Their zeros are written unless skip_dead is set: the
  // fused P3 passes read every column, the in-place inverse reads only the
  // live ones.
  constexpr int DIR0 = (MODE == PENCIL_INV) ? +1 : -1;
  bool live = true;
  if (A.live) {
    const int p = c0 + t % CB, i2 = p / A.n3, i3 = p - i2 * A.n3, h = A.live[i3];
    live = i2 <= h || i2 >= A.n2 - h;
  }
  if constexpr (MODE == PENCIL_FKI || MODE == PENCIL_FE)
    for_inputs<P0>(t, [&](int e, int row, int col) {
      v[e] = live ? load_stream<T>(&base[(long long)row * plane + col]) : mk<T>(T(0), T(0));
    });
  else
    for_inputs<P0>(t, [&](int e, int row, int col) { v[e] = base[(long long)row * plane + col]; });
  pass_compute<P0, DIR0, T>(v, tw1, t);
  exchange<P0, P1, CB, SPLIT, T>(v, smem, t);
  pass_compute<P1, DIR0, T>(v, tw1, t);

  if constexpr (MODE == PENCIL_FWD || MODE == PENCIL_INV) {
    for_outputs<P1>(t, [&](int e, int row, int col) { base[(long long)row * plane + col] = v[e]; });
    return;
  } else {
    // Coulomb kernel on the natural-order outputs (column c0 + b, k1 = row).
    // PENCIL_FE only sums the FP64 energy partials; PENCIL_FKI only scales.
    constexpr bool energy = MODE == PENCIL_FE;
    const KernelParams& kp = A.kp;
    double esum = 0.0;
    const double k0 = kp.q_zero ? *kp.k0 : 0.0;
    const typename P1::Lane l = P1::lane(t);
#pragma unroll
    for (int s = 0; s < P1::NS; ++s) {
      const int b = P1::b_of(l, s), i = P1::i_of(l, s);
      const bool act = P1::active(l, t, s);
      const int c = c0 + b;
      const int m2 = signed_index(c / A.n3, A.n2);
      const int m3 = signed_index(c - (c / A.n3) * A.n3, A.n3);
      const double gx = kp.q[0] + m2 * kp.b[1][0] + m3 * kp.b[2][0];
      const double gy = kp.q[1] + m2 * kp.b[1][1] + m3 * kp.b[2][1];
      const double gz = kp.q[2] + m2 * kp.b[1][2] + m3 * kp.b[2][2];
#pragma unroll
      for (int r = 0; r < P1::R; ++r) {
        const int m1 = signed_index(P1::out_x(i, r), N1);
        T kv;
        if constexpr (sizeof(T) == 8) {
          const double x0 = gx + m1 * kp.b[0][0], y0 = gy + m1 * kp.b[0][1], z0 = gz + m1 * kp.b[0][2];
          const double g2 = x0 * x0 + y0 * y0 + z0 * z0;
          double kk = kFourPi / g2;
          if (kp.ecut > 0.0 && g2 > kp.ecut) kk = 0.0;
          if (kp.q_zero && m1 == 0 && m2 == 0 && m3 == 0) kk = k0;
          kv = kk;
        } else {
          const float x0 = float(gx) + float(m1) * float(kp.b[0][0]);
          const float y0 = float(gy) + float(m1) * float(kp.b[0][1]);
          const float z0 = float(gz) + float(m1) * float(kp.b[0][2]);
          const float g2 = x0 * x0 + y0 * y0 + z0 * z0;
          // hardware reciprocal (1 ulp): far inside the FP32 path's error budget
          float kk = float(kFourPi) * __builtin_amdgcn_rcpf(g2);
          if (kp.ecut > 0.0) {
            const double dx = gx + m1 * kp.b[0][0], dy = gy + m1 * kp.b[0][1], dz = gz + m1 * kp.b[0][2];
            if (dx * dx + dy * dy + dz * dz > kp.ecut) kk = 0.0f;
          }
          if (kp.q_zero && m1 == 0 && m2 == 0 && m3 == 0) kk = float(k0);
          kv = kk;
        }
        cx<T>& z = v[s * P1::R + r];
        if constexpr (energy) {
          if (act) esum += double(kv * (z.x * z.x + z.y * z.y));
        } else {
          z = cscale<T>(z, kv);
        }
      }
    }
    if constexpr (energy) {
      const double tot = block_sum(esum, red);
      if (t == 0) A.epart[(long long)g * A.count + pr] = tot;
    }
    if constexpr (MODE == PENCIL_FKI) {
      exchange<P1, P0, CB, SPLIT, T>(v, smem, t);
      pass_compute<P0, +1, T>(v, tw1, t);
      exchange<P0, P1, CB, SPLIT, T>(v, smem, t);
      pass_compute<P1, +1, T>(v, tw1, t);
      // skip_dead: a 128-byte line of a row is left unwritten when every
      // column in it is dead; a partly live line is written whole (zeros
      // included), since a partial line costs the memory a read-modify-write.
      // A wave's lanes hold consecutive columns from a multiple of CB, so the
      // LINE lanes of an aligned lane group hold one line.
      bool st = true;
      if (A.live && A.skip_dead) {
        constexpr int LINE = 128 / (int)sizeof(cx<T>);
        static_assert(CB % LINE == 0 && (CB % 64 == 0 || 64 % CB == 0), "lines of whole lane groups");
        const unsigned long long m = __ballot(live);
        st = ((m >> ((threadIdx.x & 63) & ~(LINE - 1))) & ((1ull << LINE) - 1)) != 0;
      }
      if (st)
        for_outputs<P1>(t, [&](int e, int row, int col) { store_stream<T>(&base[(long long)row * plane + col], v[e]); });
    }
  }
}

template <typename T, int N1, int MODE> struct PencilCfg {
  static constexpr PencilTune P = pencil_tune(sizeof(T), N1, MODE);
  static constexpr int CB = P.cb;
  static constexpr int W = P.w;
  static constexpr bool SPLIT = P.split >= 0 ? P.split == 1 : sizeof(T) == 8 && Tile<CB>::slots(N1) * 16 > 65536;
  static constexpr int MINB = P.minb;
  static_assert(CB == pencil_tune(sizeof(T), N1).cb, "pencils per workgroup must not depend on the mode");
};

template <typename T, int N1, int CB, int W, bool SPLIT, int MODE, int MINB>
__global__ __launch_bounds__(W, MINB) void pencil_kernel(PencilArgs A) {
  using G = PencilGeom<T, N1, CB, W, SPLIT>;
  __shared__ __align__(16) unsigned char smem[G::XBYTES];
  __shared__ cx<T> tw1[N1];
  __shared__ double red[(W + 63) / 64];
  load_table<T>(tw1, A.tw1, N1);
  __syncthreads();
  pencil_body<T, N1, CB, W, SPLIT, MODE>(A, xcd_logical(blockIdx.x, gridDim.x), smem, tw1, red);
}

// ---------------------------------------------------------------------------
// Multiply-accumulate of the pair-symmetric schedule (q = 0, one orbital
// block).  The pair buffer holds v_ij in real space for a tile (i in I,
// j in J); since v_ji = conj(v_ij),
//   acc_j += sum_i f_i phi_i v_ij                 (every tile)
//   acc_i += sum_j f_j phi_j conj(v_ij)           (off-diagonal tiles only)
// Every grid point is independent: one thread per point, the tile's pairs
// in registers, each pair value read once.
// ---------------------------------------------------------------------------
struct MacArgs {
  const void* w;       // pair buffer [ti*tj][N], slot ii*tj + jj, real space
  const void* phi;     // occupied orbitals (set A) in real space [n][N]
  const double* f;     // occupations of set A
  void* acc;           // accumulators of set A [n][N] (mirror half)
  const void* phi_b;   // target orbitals (set B) and their weights (mirror
  const double* f_b;   //   half only) and accumulators (forward half); all
  void* acc_b;         //   three equal the set-A ones when one block is applied to itself
  long long N;
  int i0, j0, ti, tj, mirror;
  int tri;             // diagonal tile: pairs ii <= jj at tri_slot(ii, jj); forward ii <= jj, mirror ii < jj
};

constexpr int kMacTile = 16;  // the persistent batch schedule's and the Gamma path's tile edge

// Pair tile edge of the single-system schedules, by element size: 32 x 32
// pairs for complex FP32 (the streaming MAC then moves 1.19 N b per pair
// instead of 1.38), 16 x 16 for complex FP64, whose MAC registers would not
// hold 32 accumulators.
constexpr int pair_tile(int cplx_bytes) { return cplx_bytes == 8 ? 32 : 16; }

template <typename T>
__global__ __launch_bounds__(256) void mac_pair_kernel(MacArgs A) {
  constexpr int TILE = pair_tile((int)sizeof(cx<T>));
  const long long N = A.N;
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= N) return;
  const cx<T>* __restrict__ w = reinterpret_cast<const cx<T>*>(A.w) + p;
  const cx<T>* __restrict__ phi = reinterpret_cast<const cx<T>*>(A.phi) + p;
  // acc and acc_b are the same array when a block is applied to itself (on a
  // diagonal tile even the same rows): no __restrict__ on either
  cx<T>* acc = reinterpret_cast<cx<T>*>(A.acc) + p;
  const double* __restrict__ f = A.f;
  const cx<T>* __restrict__ phi_b = reinterpret_cast<const cx<T>*>(A.phi_b) + p;
  cx<T>* acc_b = reinterpret_cast<cx<T>*>(A.acc_b) + p;
  const double* __restrict__ f_b = A.f_b;
  const int ti = A.ti, tj = A.tj, mirror = A.mirror, tri = A.tri;
  cx<T> fphi_i[TILE], acc_i[TILE];
#pragma unroll
  for (int ii = 0; ii < TILE; ++ii) {
    if (ii < ti) fphi_i[ii] = cscale<T>(phi[(long long)(A.i0 + ii) * N], T(f[A.i0 + ii]));
    acc_i[ii] = mk<T>(T(0), T(0));
  }
  for (int jj = 0; jj < tj; ++jj) {
    const long long oj = (long long)(A.j0 + jj) * N;
    const cx<T> aj0 = acc_b[oj];
    // the forward half alone (mirror == 0) reads neither phi_b nor f_b
    const cx<T> fphi_j = mirror ? cscale<T>(phi_b[oj], T(f_b[A.j0 + jj])) : mk<T>(T(0), T(0));
    const int iend = tri ? jj + 1 : ti;  // forward: ii < iend; mirror: ii < jj on a diagonal tile
    cx<T> v[TILE];
#pragma unroll
    for (int ii = 0; ii < TILE; ++ii)
      if (ii < iend) v[ii] = load_stream<T>(&w[(long long)(tri ? tri_slot(ii, jj) : ii * tj + jj) * N]);
    T sx = aj0.x, sy = aj0.y;
#pragma unroll
    for (int ii = 0; ii < TILE; ++ii) {
      if (ii < iend) {
        const cx<T> a = cmul<T>(fphi_i[ii], v[ii]);
        sx += a.x;
        sy += a.y;
        if (mirror && (!tri || ii < jj)) {
          const cx<T> m = cmulc<T>(v[ii], fphi_j);  // conj(v) f_j phi_j
          acc_i[ii] = mk<T>(acc_i[ii].x + m.x, acc_i[ii].y + m.y);
        }
      }
    }
    acc_b[oj] = mk<T>(sx, sy);
  }
  if (mirror) {
#pragma unroll
    for (int ii = 0; ii < TILE; ++ii) {
      if (ii < ti) {
        const long long oi = (long long)(A.i0 + ii) * N;
        const cx<T> c = acc[oi];
        acc[oi] = mk<T>(c.x + acc_i[ii].x, c.y + acc_i[ii].y);
      }
    }
  }
}

// Gamma tile with v_iq = v_{i,2q} + i v_{i,2q+1} in real space in the pair
// buffer (slot ii * tj + jj): both halves in one streaming pass.  phi is the
// packed orbital array, acc the packed accumulators; a pair (i, j) adds
// f_i phi_i v_ij to acc_j when i <= j and f_j phi_j v_ij to acc_i when i < j
// (component j mod 2 of packed accumulator j / 2).  One thread per grid point
// owns every accumulator it touches, so diagonal tiles need no ordering.
template <typename T>
__global__ __launch_bounds__(256) void mac_gamma_kernel(MacArgs A, int nreal) {
  const long long N = A.N;
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= N) return;
  const cx<T>* __restrict__ w = reinterpret_cast<const cx<T>*>(A.w) + p;
  const cx<T>* __restrict__ pk = reinterpret_cast<const cx<T>*>(A.phi) + p;
  cx<T>* __restrict__ acc = reinterpret_cast<cx<T>*>(A.acc) + p;
  const double* __restrict__ f = A.f;
  const int ti = A.ti, tj = A.tj;
  T phi_i[kMacTile], mir_i[kMacTile];
#pragma unroll
  for (int ii = 0; ii < kMacTile; ++ii) {
    mir_i[ii] = T(0);
    phi_i[ii] = T(0);
    if (ii < ti) {
      const int i = A.i0 + ii;
      const cx<T> a = pk[(long long)(i >> 1) * N];
      phi_i[ii] = (i & 1) ? a.y : a.x;
    }
  }
  for (int jj = 0; jj < tj; ++jj) {
    const int q = A.j0 + jj, j0r = 2 * q, j1r = 2 * q + 1;
    const bool two = j1r < nreal;
    const long long oq = (long long)q * N;
    const cx<T> P = pk[oq];
    const cx<T> a0 = acc[oq];
    const T fj0 = T(f[j0r]), fj1 = two ? T(f[j1r]) : T(0);
    // diagonal tile: only ii < gtri_count(ti, jj) is stored, from gtri_prefix(ti, jj)
    const int iend = A.tri ? gtri_count(ti, jj) : ti;
    const int base = A.tri ? gtri_prefix(ti, jj) : jj;
    const int stride = A.tri ? 1 : tj;
    T sx = a0.x, sy = a0.y;
#pragma unroll
    for (int ii = 0; ii < kMacTile; ++ii) {
      if (ii < iend) {
        const int i = A.i0 + ii;
        const cx<T> v = load_stream<T>(&w[(long long)(base + ii * stride) * N]);
        const T fi = T(f[i]);
        const T w0 = i <= j0r ? fi : T(0), w1 = (i <= j1r && two) ? fi : T(0);
        sx += w0 * phi_i[ii] * v.x;
        sy += w1 * phi_i[ii] * v.y;
        const T m0 = i < j0r ? fj0 : T(0), m1 = (i < j1r && two) ? fj1 : T(0);
        mir_i[ii] += m0 * P.x * v.x + m1 * P.y * v.y;
      }
    }
    acc[oq] = mk<T>(sx, sy);
  }
#pragma unroll
  for (int ii = 0; ii < kMacTile; ++ii) {
    if (ii < ti) {
      const int i = A.i0 + ii;
      T* c = reinterpret_cast<T*>(acc + (long long)(i >> 1) * N) + (i & 1);
      *c += mir_i[ii];
    }
  }
}

// Mirror half only (schedule with a fused P3 that left v_ij in the pair
// buffer): acc_i += sum_j f_j phi_j conj(v_ij).  One block per (ii, i1).
template <typename T>
__global__ __launch_bounds__(256) void mac_conj_kernel(PlaneArgs A, int plane) {
  const int lid = xcd_logical(blockIdx.x, gridDim.x);
  const int i1 = lid / A.ti, ii = lid - (lid / A.ti) * A.ti;
  const long long N = A.N;
  const long long off = (long long)i1 * plane;
  const cx<T>* __restrict__ w = reinterpret_cast<const cx<T>*>(A.w) + (long long)(ii * A.tj) * N + off;
  const cx<T>* __restrict__ pb = reinterpret_cast<const cx<T>*>(A.bsrc) + (long long)A.j0 * N + off;
  cx<T>* __restrict__ pc = reinterpret_cast<cx<T>*>(A.acc) + (long long)ii * N + off;
  for (int p = threadIdx.x; p < plane; p += 256) {
    const cx<T> c = pc[p];
    T sx = c.x, sy = c.y;
    for (int jj = 0; jj < A.tj; ++jj) {
      const T fj = T(A.f[A.j0 + jj] * A.fscale);
      const cx<T> z = cmulc<T>(w[(long long)jj * N + p], pb[(long long)jj * N + p]);  // conj(v) * phi_j
      sx += fj * z.x;
      sy += fj * z.y;
    }
    pc[p] = mk<T>(sx, sy);
  }
}

// ---------------------------------------------------------------------------
// Small kernels
// ---------------------------------------------------------------------------
template <typename T>
__global__ void zero_kernel(cx<T>* p, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) p[k] = mk<T>(T(0), T(0));
}

// box[b][slot[p]] = c[b][p]  (box already zero)
template <typename T>
__global__ void scatter_kernel(const cx<T>* __restrict__ c, int ldc, const int* __restrict__ slot, int npw,
                               cx<T>* __restrict__ box, long long N) {
  const int b = blockIdx.y;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < npw; p += gridDim.x * blockDim.x)
    box[(long long)b * N + slot[p]] = c[(long long)b * ldc + p];
}

// out[j][p] = s0 * (w ? w[j0+j] : 1) * (g ? *g : 1) * box[j][slot[p]]
template <typename T>
__global__ void gather_kernel(const cx<T>* __restrict__ box, long long N, const int* __restrict__ slot, int npw,
                              cx<T>* __restrict__ out, int ldo, double s0, const double* __restrict__ w, int j0,
                              const double* __restrict__ g) {
  const int j = blockIdx.y;
  double s = s0;
  if (w) s *= w[j0 + j];
  if (g) s *= *g;
  const T st = T(s);
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < npw; p += gridDim.x * blockDim.x)
    out[(long long)j * ldo + p] = cscale<T>(box[(long long)j * N + slot[p]], st);
}

// Gamma packing of real orbitals: box[q][slot[p]] = c[2q][p] + i c[2q+1][p]
// (the second row is absent for the last q of an odd count).
template <typename T>
__global__ void scatter_pack_kernel(const cx<T>* __restrict__ c, int ldc, const int* __restrict__ slot, int npw,
                                    int nreal, cx<T>* __restrict__ box, long long N) {
  const int q = blockIdx.y;
  const bool two = 2 * q + 1 < nreal;
  const cx<T>* c0 = c + (long long)(2 * q) * ldc;
  const cx<T>* c1 = c0 + ldc;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < npw; p += gridDim.x * blockDim.x) {
    const cx<T> a = c0[p];
    const cx<T> b = two ? c1[p] : mk<T>(T(0), T(0));
    box[(long long)q * N + slot[p]] = mk<T>(a.x - b.y, a.y + b.x);
  }
}

// Unpack the transform F = FFT[acc_2q + i acc_2q+1] of two real functions on
// the sphere: FFT[acc_2q](G) = (F(G) + conj F(-G)) / 2 and
// FFT[acc_2q+1](G) = (F(G) - conj F(-G)) / (2i); rows 2q and 2q+1 of out,
// scaled by s0.
template <typename T>
__global__ void gather_unpack_kernel(const cx<T>* __restrict__ box, long long N, const int* __restrict__ slot,
                                     int npw, int n1, int n2, int n3, int nreal, cx<T>* __restrict__ out, int ldo,
                                     double s0) {
  const int q = blockIdx.y;
  const bool two = 2 * q + 1 < nreal;
  const cx<T>* F = box + (long long)q * N;
  cx<T>* o0 = out + (long long)(2 * q) * ldo;
  cx<T>* o1 = o0 + ldo;
  const T h = T(0.5 * s0);
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < npw; p += gridDim.x * blockDim.x) {
    const int s = slot[p];
    const int i3 = s % n3, i12 = s / n3;
    const int i2 = i12 % n2, i1 = i12 / n2;
    const int sm = (((n1 - i1) % n1) * n2 + (n2 - i2) % n2) * n3 + (n3 - i3) % n3;
    const cx<T> f = F[s], g = F[sm];
    o0[p] = mk<T>(h * (f.x + g.x), h * (f.y - g.y));
    if (two) o1[p] = mk<T>(h * (f.y + g.y), h * (g.x - f.x));
  }
}

// part[b] = g[b] Re sum_p conj(c[b][p]) v[b][p]  (one block per band, FP64 sum;
// g null: weight 1).  With v = V_x psi, 1/2 sum_b part[b] is the exchange
// energy of the block; with v = dE/d conj(c) (weights already inside),
// 1/2 sum_b part[b] is E itself (E has degree 2 in conj(c)).
template <typename T>
__global__ void band_dot_kernel(const cx<T>* __restrict__ c, int ldc, const cx<T>* __restrict__ v, int ldv, int npw,
                                const double* __restrict__ g, double* __restrict__ part) {
  __shared__ double red[4];
  const int b = blockIdx.x;
  const cx<T>* cb = c + (long long)b * ldc;
  const cx<T>* vb = v + (long long)b * ldv;
  double s = 0.0;
  for (int p = threadIdx.x; p < npw; p += blockDim.x) {
    const cx<T> x = cb[p], y = vb[p];
    s += double(x.x) * double(y.x) + double(x.y) * double(y.y);
  }
  const double tot = block_sum(s, red);
  if (threadIdx.x == 0) part[b] = g ? g[b] * tot : tot;
}

// Band force on the sphere:
//   out[j][p] = -w[j0+j] * (1/2 |k+G_p|^2 c[j][p] + box[j][slot[p]] / N)
struct ForceArgs {
  const void* box;     // [nj][N]: FFT[V psi_j], unnormalised
  long long N;
  const int* slot;
  int npw;
  const void* c;       // [*][ldc] sphere coefficients (row j0 + j)
  int ldc;
  void* out;           // [*][ldo] (row j0 + j)
  int ldo;
  const double* w;
  int j0;
  double b[3][3];      // reciprocal vectors (rows)
  double k[3];
  int n1, n2, n3;
};

template <typename T>
__global__ void force_gather_kernel(ForceArgs A) {
  const int j = blockIdx.y;
  const double wj = A.w[A.j0 + j];
  const cx<T>* box = reinterpret_cast<const cx<T>*>(A.box) + (long long)j * A.N;
  const cx<T>* c = reinterpret_cast<const cx<T>*>(A.c) + (long long)(A.j0 + j) * A.ldc;
  cx<T>* out = reinterpret_cast<cx<T>*>(A.out) + (long long)(A.j0 + j) * A.ldo;
  const double inv_n = 1.0 / double(A.N);
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < A.npw; p += gridDim.x * blockDim.x) {
    const int s = A.slot[p];
    const int i3 = s % A.n3, i12 = s / A.n3;
    const int i2 = i12 % A.n2, i1 = i12 / A.n2;
    const int m1 = signed_index(i1, A.n1), m2 = signed_index(i2, A.n2), m3 = signed_index(i3, A.n3);
    double g2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double ga = A.k[a] + m1 * A.b[0][a] + m2 * A.b[1][a] + m3 * A.b[2][a];
      g2 += ga * ga;
    }
    const cx<T> v = box[s], cp = c[p];
    const T kin = T(0.5 * g2), sv = T(inv_n), mw = T(-wj);
    out[p] = mk<T>(mw * (kin * cp.x + sv * v.x), mw * (kin * cp.y + sv * v.y));
  }
}

}  // namespace fockx
