// Batched form: the band-pair work of several systems (uneven cubic grids and
// band counts) in one persistent launch.
//
// The work is a list of segments, one per (system, pair tile, stage):
//   P1   pair density + forward plane FFT     units: pairs x planes
//   P2   pencil FFT + Coulomb kernel + inverse  units: pairs x column groups
//   P3   inverse plane FFT in place             units: pairs x planes
//   MAC  multiply-accumulate of both mirror images (pair-symmetric schedule)
//        units: chunks of grid points
// Units are numbered consecutively across segments in a topological order:
// every segment's dependencies precede it.  A block takes a ticket of K
// consecutive units from a device counter, waits until the dependencies of
// each unit's segment are complete, runs the unit, and adds to the segment's
// done counter.  Tickets are taken only by running blocks, in order, so every
// wait is on work already held by a running block: the launch cannot deadlock
// whatever the grid size.  Waits are bounded in time (the device's constant
// wall clock); a block whose wait exceeds the bound raises the abort flag,
// and every block stops taking work once it is set, so the launch always
// drains.
#pragma once

#include "fock_kernels.h"

namespace fockx {

constexpr int kBatchW = 576;  // multiple of every lane-fastest extent for n in {24,48,64,72,96}
constexpr int kMaxDeps = 2;

struct BatchSys {
  void* phi;          // [nb][N] orbitals in real space
  void* acc;          // [nb][N] accumulators
  const double* f;    // [nb] occupations
  const void* tw;     // twiddle table of length n (cubic grid)
  KernelParams kp;
  long long N;
  int n, nb, ngroups;
};

enum BatchStage : int { BS_P1 = 0, BS_P2 = 1, BS_P3 = 2, BS_MAC = 3 };

struct BatchSeg {
  long long start;    // first unit
  int units;
  int sys, stage, slot;
  int i0, j0, ti, tj;
  int dep[kMaxDeps];  // segment indices (-1: none); each must reach its unit count
};

struct BatchArgs {
  const BatchSys* sys;
  const BatchSeg* seg;
  int nseg;
  long long total_units;
  int units_per_ticket;
  void* const* slots;            // pair buffers
  unsigned long long* ticket;    // next unit to hand out
  int* done;                     // per segment: finished units
  int* abort_flag;               // set by a block whose wait exceeded the bound
  const long long* wait_ticks;   // device: bound on one dependency wait, wall-clock ticks
};

// Multiply-accumulate of one chunk of grid points (the pair-symmetric
// schedule's MAC, as mac_pair_kernel), the tile's occupied index taken in two
// halves of up to 8 to bound the registers of the persistent kernel.
template <typename T>
__device__ __forceinline__ void batch_mac_unit(const MacArgs& A, long long p0) {
  constexpr int H = kMacTile / 2;
  const long long N = A.N;
  const long long p = p0 + threadIdx.x;
  if (p >= N) return;
  const cx<T>* __restrict__ w = reinterpret_cast<const cx<T>*>(A.w) + p;
  const cx<T>* __restrict__ phi = reinterpret_cast<const cx<T>*>(A.phi) + p;
  cx<T>* __restrict__ acc = reinterpret_cast<cx<T>*>(A.acc) + p;
  const double* __restrict__ f = A.f;
  const int ti = A.ti, tj = A.tj, mirror = A.mirror;
  for (int h0 = 0; h0 < ti; h0 += H) {
    cx<T> fphi_i[H], acc_i[H];
#pragma unroll
    for (int ii = 0; ii < H; ++ii) {
      if (h0 + ii < ti) fphi_i[ii] = cscale<T>(phi[(long long)(A.i0 + h0 + ii) * N], T(f[A.i0 + h0 + ii]));
      acc_i[ii] = mk<T>(T(0), T(0));
    }
    for (int jj = 0; jj < tj; ++jj) {
      const long long oj = (long long)(A.j0 + jj) * N;
      const cx<T> aj0 = acc[oj];
      const cx<T> fphi_j = cscale<T>(phi[oj], T(f[A.j0 + jj]));
      cx<T> v[H];
#pragma unroll
      for (int ii = 0; ii < H; ++ii)
        if (h0 + ii < ti) v[ii] = w[(long long)((h0 + ii) * tj + jj) * N];
      T sx = aj0.x, sy = aj0.y;
#pragma unroll
      for (int ii = 0; ii < H; ++ii) {
        if (h0 + ii < ti) {
          const cx<T> a = cmul<T>(fphi_i[ii], v[ii]);
          sx += a.x;
          sy += a.y;
          if (mirror) {
            const cx<T> m = cmulc<T>(v[ii], fphi_j);
            acc_i[ii] = mk<T>(acc_i[ii].x + m.x, acc_i[ii].y + m.y);
          }
        }
      }
      acc[oj] = mk<T>(sx, sy);
    }
    if (mirror) {
#pragma unroll
      for (int ii = 0; ii < H; ++ii) {
        if (h0 + ii < ti) {
          const long long oi = (long long)(A.i0 + h0 + ii) * N;
          const cx<T> c = acc[oi];
          acc[oi] = mk<T>(c.x + acc_i[ii].x, c.y + acc_i[ii].y);
        }
      }
    }
  }
}

template <typename T, int NN> struct BatchShape {
  static constexpr int CB = pencil_tune(sizeof(T), NN).cb;
  static constexpr bool PSPLIT = sizeof(T) == 8 && plane_slots<NN, plane_tile_pad<T, NN>()>(NN) * 16 > 65536;
  static constexpr bool CSPLIT = sizeof(T) == 8 && Tile<CB>::slots(NN) * 16 > 65536;
  static constexpr int XBYTES_P = PlaneGeom<T, NN, NN, kBatchW, PSPLIT>::XBYTES;
  static constexpr int XBYTES_C = PencilGeom<T, NN, CB, kBatchW, CSPLIT>::XBYTES;
  static constexpr int XBYTES = XBYTES_P > XBYTES_C ? XBYTES_P : XBYTES_C;
};

// Each stage body is its own (non-inlined) function so that it gets its own
// register allocation; the dispatcher keeps only a handful of values live.
template <typename T, int NN, int OCC>
__device__ __noinline__ void batch_plane_unit(void* slot, const BatchSys* Sp, const BatchSeg* gp, int u,
                                              unsigned char* smem, const cx<T>* tw) {
  using Sh = BatchShape<T, NN>;
  const BatchSys& S = *Sp;
  const BatchSeg& g = *gp;
  PlaneArgs A{};
  A.a = S.phi;
  A.bsrc = S.phi;
  A.w = slot;
  A.x = slot;
  A.N = S.N;
  A.i0 = g.i0;
  A.j0 = g.j0;
  A.ti = g.ti;
  A.tj = g.tj;
  A.n1 = NN;
  A.nb = g.ti * g.tj;
  if (g.stage == BS_P1)
    plane_body<T, NN, NN, kBatchW, Sh::PSPLIT, PLANE_PAIR_FWD>(A, u, smem, tw, tw);
  else
    plane_body<T, NN, NN, kBatchW, Sh::PSPLIT, PLANE_INV>(A, u, smem, tw, tw);
}

template <typename T, int NN, int OCC>
__device__ __noinline__ void batch_pencil_unit(void* slot, const BatchSys* Sp, const BatchSeg* gp, int u,
                                               unsigned char* smem, const cx<T>* tw, double* red) {
  using Sh = BatchShape<T, NN>;
  PencilArgs A{};
  A.x = slot;
  A.epart = nullptr;
  A.kp = Sp->kp;
  A.N = Sp->N;
  A.n2 = NN;
  A.n3 = NN;
  A.count = gp->ti * gp->tj;
  pencil_body<T, NN, Sh::CB, kBatchW, Sh::CSPLIT, PENCIL_FKI>(A, u, smem, tw, red);
}

template <typename T, int OCC>
__device__ __noinline__ void batch_mac_call(void* slot, const BatchSys* Sp, const BatchSeg* gp, int u) {
  MacArgs A{};
  A.w = slot;
  A.phi = Sp->phi;
  A.f = Sp->f;
  A.acc = Sp->acc;
  A.N = Sp->N;
  A.i0 = gp->i0;
  A.j0 = gp->j0;
  A.ti = gp->ti;
  A.tj = gp->tj;
  A.mirror = gp->i0 != gp->j0;
  batch_mac_unit<T>(A, (long long)u * kBatchW);
}

template <typename T, int NN, int OCC>
__device__ __forceinline__ void batch_run_unit(const BatchArgs& B, const BatchSeg& g, const BatchSys& S, int u,
                                               unsigned char* smem, const cx<T>* tw, double* red) {
  void* slot = B.slots[g.slot];
  if (g.stage == BS_P1 || g.stage == BS_P3)
    batch_plane_unit<T, NN, OCC>(slot, &S, &g, u, smem, tw);
  else if (g.stage == BS_P2)
    batch_pencil_unit<T, NN, OCC>(slot, &S, &g, u, smem, tw, red);
  else
    batch_mac_call<T, OCC>(slot, &S, &g, u);
}

// Segment holding `unit`.  A block's tickets only move forward, so the search
// starts at the block's previous segment and steps ahead.
__device__ __forceinline__ int batch_find_seg(const BatchSeg* seg, int nseg, long long unit, int from) {
  int g = from;
  while (g + 1 < nseg && seg[g + 1].start <= unit) ++g;
  return g;
}

template <typename T, int OCC>
__device__ __forceinline__ void batch_kernel_body(const BatchArgs& B) {
  constexpr int XB = BatchShape<T, 96>::XBYTES > BatchShape<T, 72>::XBYTES ? BatchShape<T, 96>::XBYTES
                                                                            : BatchShape<T, 72>::XBYTES;
  __shared__ __align__(16) unsigned char smem[XB];
  __shared__ cx<T> tw[128];
  __shared__ double red[(kBatchW + 63) / 64];
  __shared__ long long s_first;
  __shared__ int s_go;
  int tw_n = 0;
  int last_seg = 0;  // meaningful in thread 0 only
  const int t = threadIdx.x;
  for (;;) {
    if (t == 0) {
      long long first = -1;
      if (__hip_atomic_load(B.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
        const unsigned long long k = __hip_atomic_fetch_add(B.ticket, (unsigned long long)B.units_per_ticket,
                                                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((long long)k < B.total_units) first = (long long)k;
      }
      s_first = first;
    }
    __syncthreads();
    const long long first = s_first;
    if (first < 0) return;
    const long long last = first + B.units_per_ticket < B.total_units ? first + B.units_per_ticket : B.total_units;
    long long unit = first;
    while (unit < last) {
      // the segment of this unit, and how many of the ticket's units it covers
      __shared__ int s_seg;
      if (t == 0) {
        const int gi = batch_find_seg(B.seg, B.nseg, unit, last_seg);
        last_seg = gi;
        int go = 1;
        for (int d = 0; d < kMaxDeps && go; ++d) {
          const int dep = B.seg[gi].dep[d];
          if (dep < 0) continue;
          const int need = B.seg[dep].units;
          const long long limit = *B.wait_ticks;
          const long long t_wait = wall_clock64();
          while (__hip_atomic_load(&B.done[dep], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
            if (__hip_atomic_load(B.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                wall_clock64() - t_wait > limit) {
              __hip_atomic_store(B.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              go = 0;
              break;
            }
            __builtin_amdgcn_s_sleep(2);
          }
        }
        s_seg = gi;
        s_go = go;
      }
      __syncthreads();
      if (!s_go) return;
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const BatchSeg g = B.seg[s_seg];
      const BatchSys S = B.sys[g.sys];
      const long long seg_end = g.start + g.units;
      const long long stop = last < seg_end ? last : seg_end;
      if (S.n != tw_n) {
        __syncthreads();
        load_table<T>(tw, S.tw, S.n);
        tw_n = S.n;
        __syncthreads();
      }
      for (long long x = unit; x < stop; ++x) {
        const int u = (int)(x - g.start);
        switch (S.n) {
          case 24: batch_run_unit<T, 24, OCC>(B, g, S, u, smem, tw, red); break;
          case 48: batch_run_unit<T, 48, OCC>(B, g, S, u, smem, tw, red); break;
          case 64: batch_run_unit<T, 64, OCC>(B, g, S, u, smem, tw, red); break;
          case 72: batch_run_unit<T, 72, OCC>(B, g, S, u, smem, tw, red); break;
          case 96: batch_run_unit<T, 96, OCC>(B, g, S, u, smem, tw, red); break;
          default: break;
        }
        __syncthreads();
      }
      if (t == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(&B.done[s_seg], (int)(stop - unit), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      unit = stop;
    }
  }
}


// Register budget variants: one persistent block per compute unit (up to 168
// VGPRs, no spills) or two (at most 5 waves per SIMD: 96 VGPRs, some spills).
// The autotuner times both.
template <typename T>
__global__ __launch_bounds__(kBatchW) void batch_kernel_occ1(BatchArgs B) {
  batch_kernel_body<T, 1>(B);
}
template <typename T>
__global__ __launch_bounds__(kBatchW) __attribute__((amdgpu_waves_per_eu(5, 8))) void batch_kernel_occ2(BatchArgs B) {
  batch_kernel_body<T, 2>(B);
}

}  // namespace fockx
