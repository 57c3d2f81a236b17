// Instantiates every plane / pencil kernel for one real type FX_T.
#include "fock_launch.h"

namespace fockx {

namespace {
template <int MODE, int N2, int N3>
hipError_t plane_go(const PlaneArgs& a, int nblocks, hipStream_t s) {
  using T = FX_T;
  using C = PlaneCfg<T, N2, N3, MODE>;
  hipLaunchKernelGGL((plane_kernel<T, N2, N3, C::W, C::SPLIT, MODE, C::MINB>), dim3(nblocks), dim3(C::W), 0, s, a);
  return hipGetLastError();
}
template <int N2, int N3>
hipError_t plane_mode(int mode, const PlaneArgs& a, int nblocks, hipStream_t s) {
  switch (mode) {
    case PLANE_PAIR_FWD: return plane_go<PLANE_PAIR_FWD, N2, N3>(a, nblocks, s);
    case PLANE_INV_MAC: return plane_go<PLANE_INV_MAC, N2, N3>(a, nblocks, s);
    case PLANE_FWD: return plane_go<PLANE_FWD, N2, N3>(a, nblocks, s);
    case PLANE_INV: return plane_go<PLANE_INV, N2, N3>(a, nblocks, s);
    case PLANE_INV_MAC_MIR: return plane_go<PLANE_INV_MAC_MIR, N2, N3>(a, nblocks, s);
    case PLANE_DENS: return plane_go<PLANE_DENS, N2, N3>(a, nblocks, s);
    case PLANE_VMUL: return plane_go<PLANE_VMUL, N2, N3>(a, nblocks, s);
    case PLANE_PAIR_FWD_G: return plane_go<PLANE_PAIR_FWD_G, N2, N3>(a, nblocks, s);
    case PLANE_INV_MAC_G: return plane_go<PLANE_INV_MAC_G, N2, N3>(a, nblocks, s);
    case PLANE_INV_MAC_MIR_G: return plane_go<PLANE_INV_MAC_MIR_G, N2, N3>(a, nblocks, s);
  }
  return hipErrorInvalidValue;
}
template <int MODE, int N1>
hipError_t pencil_go(const PencilArgs& a, int nblocks, hipStream_t s) {
  using T = FX_T;
  using C = PencilCfg<T, N1, MODE>;
  hipLaunchKernelGGL((pencil_kernel<T, N1, C::CB, C::W, C::SPLIT, MODE, C::MINB>), dim3(nblocks), dim3(C::W), 0, s, a);
  return hipGetLastError();
}
template <int N1>
hipError_t pencil_mode(int mode, const PencilArgs& a, int nblocks, hipStream_t s) {
  switch (mode) {
    case PENCIL_FKI: return pencil_go<PENCIL_FKI, N1>(a, nblocks, s);
    case PENCIL_FE: return pencil_go<PENCIL_FE, N1>(a, nblocks, s);
    case PENCIL_FWD: return pencil_go<PENCIL_FWD, N1>(a, nblocks, s);
    case PENCIL_INV: return pencil_go<PENCIL_INV, N1>(a, nblocks, s);
  }
  return hipErrorInvalidValue;
}
}  // namespace

template <>
hipError_t launch_plane<FX_T>(int mode, int n2, int n3, const PlaneArgs& a, int nblocks, hipStream_t s) {
#define FX_PLANE(A, B) \
  if (n2 == A && n3 == B) return plane_mode<A, B>(mode, a, nblocks, s);
  FX_PLANE(24, 24)
  FX_PLANE(48, 48)
  FX_PLANE(48, 64)
  FX_PLANE(64, 64)
  FX_PLANE(72, 72)
  FX_PLANE(96, 96)
  FX_PLANE(96, 128)
#undef FX_PLANE
  return hipErrorInvalidValue;
}

template <>
hipError_t launch_pencil<FX_T>(int mode, int n1, const PencilArgs& a, int nblocks, hipStream_t s) {
  switch (n1) {
    case 24: return pencil_mode<24>(mode, a, nblocks, s);
    case 48: return pencil_mode<48>(mode, a, nblocks, s);
    case 64: return pencil_mode<64>(mode, a, nblocks, s);
    case 72: return pencil_mode<72>(mode, a, nblocks, s);
    case 96: return pencil_mode<96>(mode, a, nblocks, s);
    case 128: return pencil_mode<128>(mode, a, nblocks, s);
  }
  return hipErrorInvalidValue;
}

template <>
hipError_t launch_batch<FX_T>(const BatchArgs& a, int occ, int grid, hipStream_t s) {
  if (occ == 2)
    hipLaunchKernelGGL(batch_kernel_occ2<FX_T>, dim3(grid), dim3(kBatchW), 0, s, a);
  else
    hipLaunchKernelGGL(batch_kernel_occ1<FX_T>, dim3(grid), dim3(kBatchW), 0, s, a);
  return hipGetLastError();
}

template <>
int batch_blocks_per_cu<FX_T>(int occ) {
  int n = 0;
  hipError_t e = occ == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel_occ2<FX_T>, kBatchW, 0)
                          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel_occ1<FX_T>, kBatchW, 0);
  if (e != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

template <>
hipError_t launch_mac_conj<FX_T>(const PlaneArgs& a, int plane, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(mac_conj_kernel<FX_T>, dim3(nblocks), dim3(256), 0, s, a, plane);
  return hipGetLastError();
}

template <>
hipError_t launch_mac_pair<FX_T>(const MacArgs& a, hipStream_t s) {
  const long long blocks = (a.N + 255) / 256;
  hipLaunchKernelGGL(mac_pair_kernel<FX_T>, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <>
hipError_t launch_zero<FX_T>(void* p, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  long long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(zero_kernel<FX_T>, dim3((unsigned)blocks), dim3(256), 0, s, reinterpret_cast<cx<FX_T>*>(p), n);
  return hipGetLastError();
}

template <>
hipError_t launch_scatter<FX_T>(const void* c, int ldc, const int* slot, int npw, int nb, void* box, long long N,
                                hipStream_t s) {
  if (nb <= 0 || npw <= 0) return hipSuccess;
  const int bx = (npw + 255) / 256;
  hipLaunchKernelGGL(scatter_kernel<FX_T>, dim3(bx, nb), dim3(256), 0, s, reinterpret_cast<const cx<FX_T>*>(c), ldc,
                     slot, npw, reinterpret_cast<cx<FX_T>*>(box), N);
  return hipGetLastError();
}

template <>
hipError_t launch_gather<FX_T>(const void* box, long long N, const int* slot, int npw, int nj, void* out, int ldo,
                               double s0, const double* w, int j0, const double* g, hipStream_t s) {
  if (nj <= 0 || npw <= 0) return hipSuccess;
  const int bx = (npw + 255) / 256;
  hipLaunchKernelGGL(gather_kernel<FX_T>, dim3(bx, nj), dim3(256), 0, s, reinterpret_cast<const cx<FX_T>*>(box), N,
                     slot, npw, reinterpret_cast<cx<FX_T>*>(out), ldo, s0, w, j0, g);
  return hipGetLastError();
}

template <>
hipError_t launch_scatter_pack<FX_T>(const void* c, int ldc, const int* slot, int npw, int nreal, void* box,
                                     long long N, hipStream_t s) {
  const int m = (nreal + 1) / 2;
  if (m <= 0 || npw <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_pack_kernel<FX_T>, dim3((npw + 255) / 256, m), dim3(256), 0, s,
                     reinterpret_cast<const cx<FX_T>*>(c), ldc, slot, npw, nreal, reinterpret_cast<cx<FX_T>*>(box), N);
  return hipGetLastError();
}

template <>
hipError_t launch_gather_unpack<FX_T>(const void* box, long long N, const int* slot, int npw, const int n[3],
                                      int nreal, void* out, int ldo, double s0, hipStream_t s) {
  const int m = (nreal + 1) / 2;
  if (m <= 0 || npw <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_unpack_kernel<FX_T>, dim3((npw + 255) / 256, m), dim3(256), 0, s,
                     reinterpret_cast<const cx<FX_T>*>(box), N, slot, npw, n[0], n[1], n[2], nreal,
                     reinterpret_cast<cx<FX_T>*>(out), ldo, s0);
  return hipGetLastError();
}

template <>
hipError_t launch_mac_gamma<FX_T>(const MacArgs& a, int nreal, hipStream_t s) {
  const long long blocks = (a.N + 255) / 256;
  hipLaunchKernelGGL(mac_gamma_kernel<FX_T>, dim3((unsigned)blocks), dim3(256), 0, s, a, nreal);
  return hipGetLastError();
}

template <>
hipError_t launch_band_dot<FX_T>(const void* c, int ldc, const void* v, int ldv, int npw, const double* g, int nb,
                                 double* part, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(band_dot_kernel<FX_T>, dim3(nb), dim3(256), 0, s, reinterpret_cast<const cx<FX_T>*>(c), ldc,
                     reinterpret_cast<const cx<FX_T>*>(v), ldv, npw, g, part);
  return hipGetLastError();
}

template <>
hipError_t launch_force_gather<FX_T>(const ForceArgs& a, int nj, hipStream_t s) {
  if (nj <= 0 || a.npw <= 0) return hipSuccess;
  const int bx = (a.npw + 255) / 256;
  hipLaunchKernelGGL(force_gather_kernel<FX_T>, dim3(bx, nj), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace fockx
