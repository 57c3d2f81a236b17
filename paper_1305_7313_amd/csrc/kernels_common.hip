// Type-independent kernels: energy reductions, Gygi-Baldereschi constant.
#include <cstring>

#include "fock_launch.h"

namespace fockx {

// Per tile: sum_{pairs} f_i g_j sum_groups epart -> tile_e[tile]   (one block, fixed order)
// sym: the tile stands for both orders of each pair (one orbital block, q = 0,
// sum_G K |rho_ji|^2 = sum_G K |rho_ij|^2): weight f_i g_j + f_j g_i, and in a
// diagonal tile (i0 == j0) only ii < jj counts twice, ii == jj once.
__global__ void energy_tile_kernel(const double* __restrict__ epart, int ngroups, const double* __restrict__ f,
                                   const double* __restrict__ g, int i0, int j0, int ti, int tj, int sym,
                                   int tri, double escale, double* __restrict__ tile_e) {
  __shared__ double red[16];
  double acc = 0.0;
  // tri: a diagonal tile holding only the pairs ii <= jj, at tri_slot(ii, jj)
  const int np = tri ? tri_slot(0, ti) : ti * tj;
  for (int pr = threadIdx.x; pr < np; pr += blockDim.x) {
    int ii, jj;
    if (tri) {
      jj = 0;
      while (tri_slot(0, jj + 1) <= pr) ++jj;
      ii = pr - tri_slot(0, jj);
    } else {
      ii = pr / tj;
      jj = pr - ii * tj;
    }
    const int i = i0 + ii, j = j0 + jj;
    double wgt = f[i] * g[j];
    if (sym) {
      if (i0 == j0) wgt = ii < jj ? wgt + f[j] * g[i] : (ii == jj ? wgt : 0.0);
      else wgt += f[j] * g[i];
    }
    if (wgt == 0.0) continue;
    // group-major partials (consecutive threads read consecutive words), four
    // independent partial sums so that the loads overlap; fixed combination order
    const double* e = epart + pr;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int k = 0;
    for (; k + 4 <= ngroups; k += 4) {
      s0 += e[(long long)k * np];
      s1 += e[(long long)(k + 1) * np];
      s2 += e[(long long)(k + 2) * np];
      s3 += e[(long long)(k + 3) * np];
    }
    for (; k < ngroups; ++k) s0 += e[(long long)k * np];
    acc += wgt * ((s0 + s1) + (s2 + s3));
  }
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) *tile_e = escale * tot;
}

// ex = scale * sum_t tile_e[t]   (one thread, fixed order)
__global__ void energy_final_kernel(const double* __restrict__ tile_e, int ntiles, double scale, double* ex) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < ntiles; ++k) s += tile_e[k];
    *ex = scale * s;
  }
}

// Gygi-Baldereschi lattice sum: partial[block] = sum over (q in mesh, G in box, q+G != 0)
// of 4 pi exp(-alpha |q+G|^2) / |q+G|^2.
__global__ void gb_partial_kernel(KernelParams kp, int n1, int n2, int n3, int nq1, int nq2, int nq3, double alpha,
                                  double* partial) {
  __shared__ double red[16];
  const long long N = (long long)n1 * n2 * n3;
  const long long total = N * nq1 * nq2 * nq3;
  double acc = 0.0;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < total;
       k += (long long)gridDim.x * blockDim.x) {
    const long long iq = k / N, ib = k - (k / N) * N;
    const int s3 = (int)(iq % nq3), s2 = (int)((iq / nq3) % nq2), s1 = (int)(iq / ((long long)nq3 * nq2));
    const int i3 = (int)(ib % n3), i2 = (int)((ib / n3) % n2), i1 = (int)(ib / ((long long)n3 * n2));
    const double f1 = signed_index(i1, n1) + double(s1) / nq1;
    const double f2 = signed_index(i2, n2) + double(s2) / nq2;
    const double f3 = signed_index(i3, n3) + double(s3) / nq3;
    const double gx = f1 * kp.b[0][0] + f2 * kp.b[1][0] + f3 * kp.b[2][0];
    const double gy = f1 * kp.b[0][1] + f2 * kp.b[1][1] + f3 * kp.b[2][1];
    const double gz = f1 * kp.b[0][2] + f2 * kp.b[1][2] + f3 * kp.b[2][2];
    const double g2 = gx * gx + gy * gy + gz * gz;
    if (iq == 0 && ib == 0) continue;
    acc += kFourPi * exp(-alpha * g2) / g2;
  }
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ void gb_final_kernel(const double* partial, int nparts, double head, double* k0) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < nparts; ++k) s += partial[k];
    *k0 = head - s;
  }
}

__global__ void set_scalar_kernel(double* p, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}


bool plane_supported(int n2, int n3) {
  return (n2 == 24 && n3 == 24) || (n2 == 48 && n3 == 48) || (n2 == 48 && n3 == 64) || (n2 == 64 && n3 == 64) ||
         (n2 == 72 && n3 == 72) || (n2 == 96 && n3 == 96) || (n2 == 96 && n3 == 128);
}
bool pencil_supported(int n1) {
  return n1 == 24 || n1 == 48 || n1 == 64 || n1 == 72 || n1 == 96 || n1 == 128;
}
int pencil_columns(int n1, int tbytes) {
  if (!pencil_supported(n1)) return 0;
  return pencil_tune(tbytes, n1).cb;
}

hipError_t launch_energy_tile(const double* epart, int ngroups, const double* f, const double* g, int i0, int j0,
                              int ti, int tj, int sym, int tri, double escale, double* tile_e, hipStream_t s) {
  hipLaunchKernelGGL(energy_tile_kernel, dim3(1), dim3(256), 0, s, epart, ngroups, f, g, i0, j0, ti, tj, sym, tri,
                     escale, tile_e);
  return hipGetLastError();
}

// rho[r] = sum_g part[g][r]  (fixed order: bitwise reproducible)
__global__ void group_sum_kernel(const double* __restrict__ part, int ngrp, long long N, double* __restrict__ rho) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += stride) {
    double s = 0.0;
    for (int g = 0; g < ngrp; ++g) s += part[(long long)g * N + r];
    rho[r] = s;
  }
}

hipError_t launch_group_sum(const double* part, int ngrp, long long N, double* rho, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  long long blocks = (N + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(group_sum_kernel, dim3((unsigned)blocks), dim3(256), 0, s, part, ngrp, N, rho);
  return hipGetLastError();
}

hipError_t launch_energy_final(const double* tile_e, int ntiles, double scale, double* ex, hipStream_t s) {
  hipLaunchKernelGGL(energy_final_kernel, dim3(1), dim3(64), 0, s, tile_e, ntiles, scale, ex);
  return hipGetLastError();
}

hipError_t launch_gb(const KernelParams& kp, const int n[3], const int nq[3], double alpha, double head,
                     double* partial, int nparts, double* k0, hipStream_t s) {
  hipLaunchKernelGGL(gb_partial_kernel, dim3(nparts), dim3(256), 0, s, kp, n[0], n[1], n[2], nq[0], nq[1], nq[2],
                     alpha, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gb_final_kernel, dim3(1), dim3(64), 0, s, partial, nparts, head, k0);
  return hipGetLastError();
}

// Zeroes the batch scheduler state (a kernel, so that a captured graph replays it).
__global__ void batch_reset_kernel(unsigned long long* ticket, int* done, int nseg, int* abort_flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    *ticket = 0ull;
    *abort_flag = 0;
  }
  for (int k = i; k < nseg; k += gridDim.x * blockDim.x) done[k] = 0;
}

hipError_t launch_batch_reset(unsigned long long* ticket, int* done, int nseg, int* abort_flag, hipStream_t s) {
  const int blocks = (nseg + 255) / 256 > 0 ? ((nseg + 255) / 256 < 1024 ? (nseg + 255) / 256 : 1024) : 1;
  hipLaunchKernelGGL(batch_reset_kernel, dim3(blocks), dim3(256), 0, s, ticket, done, nseg, abort_flag);
  return hipGetLastError();
}

// Host bytes carried to the device as kernel arguments, a chunk per launch:
// stream ordered, no staging buffer, nothing for the caller to keep alive.
constexpr int kPutWords = 512;
struct PutChunk {
  int n;
  uint32_t w[kPutWords];
};

__global__ void put_words_kernel(uint32_t* dst, PutChunk c) {
  for (int k = threadIdx.x; k < c.n; k += blockDim.x) dst[k] = c.w[k];
}

hipError_t launch_put_words(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes % 4 != 0) return hipErrorInvalidValue;
  const size_t words = bytes / 4;
  const unsigned char* from = static_cast<const unsigned char*>(src);
  for (size_t w0 = 0; w0 < words; w0 += kPutWords) {
    PutChunk c;
    c.n = (int)(words - w0 < (size_t)kPutWords ? words - w0 : (size_t)kPutWords);
    std::memcpy(c.w, from + 4 * w0, 4 * (size_t)c.n);
    hipLaunchKernelGGL(put_words_kernel, dim3(1), dim3(256), 0, s, static_cast<uint32_t*>(dst) + w0, c);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_set_scalar(double* p, double v, hipStream_t s) {
  hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

}  // namespace fockx
