// Host-side launchers of the device kernels (one instantiation per dtype).
#pragma once

#include <hip/hip_runtime.h>

#include "fock_kernels.h"
#include "batch_kernel.h"

namespace fockx {

bool plane_supported(int n2, int n3);
bool pencil_supported(int n1);
int pencil_columns(int n1, int tbytes);  // columns per pencil workgroup

template <typename T> hipError_t launch_plane(int mode, int n2, int n3, const PlaneArgs& a, int nblocks, hipStream_t s);
template <typename T> hipError_t launch_pencil(int mode, int n1, const PencilArgs& a, int nblocks, hipStream_t s);
template <typename T> hipError_t launch_zero(void* p, long long n, hipStream_t s);
template <typename T> hipError_t launch_mac_pair(const MacArgs& a, hipStream_t s);
template <typename T> hipError_t launch_mac_conj(const PlaneArgs& a, int plane, int nblocks, hipStream_t s);
template <typename T>
hipError_t launch_scatter(const void* c, int ldc, const int* slot, int npw, int nb, void* box, long long N, hipStream_t s);
template <typename T>
hipError_t launch_gather(const void* box, long long N, const int* slot, int npw, int nj, void* out, int ldo, double s0,
                         const double* w, int j0, const double* g, hipStream_t s);

template <typename T>
hipError_t launch_scatter_pack(const void* c, int ldc, const int* slot, int npw, int nreal, void* box, long long N,
                               hipStream_t s);
template <typename T>
hipError_t launch_gather_unpack(const void* box, long long N, const int* slot, int npw, const int n[3], int nreal,
                                void* out, int ldo, double s0, hipStream_t s);
template <typename T> hipError_t launch_mac_gamma(const MacArgs& a, int nreal, hipStream_t s);
template <typename T>
hipError_t launch_band_dot(const void* c, int ldc, const void* v, int ldv, int npw, const double* g, int nb,
                           double* part, hipStream_t s);
template <typename T> hipError_t launch_force_gather(const ForceArgs& a, int nj, hipStream_t s);
hipError_t launch_group_sum(const double* part, int ngrp, long long N, double* rho, hipStream_t s);

hipError_t launch_energy_tile(const double* epart, int ngroups, const double* f, const double* g, int i0, int j0, int ti,
                              int tj, int sym, int tri, double escale, double* tile_e, hipStream_t s);
hipError_t launch_energy_final(const double* tile_e, int ntiles, double scale, double* ex, hipStream_t s);
hipError_t launch_gb(const KernelParams& kp, const int n[3], const int nq[3], double alpha, double head,
                     double* partial, int nparts, double* k0, hipStream_t s);
hipError_t launch_set_scalar(double* p, double v, hipStream_t s);
// Copies `bytes` (a multiple of 4) of host memory to dst through kernel arguments.
hipError_t launch_put_words(void* dst, const void* src, size_t bytes, hipStream_t s);
template <typename T> hipError_t launch_batch(const BatchArgs& a, int occ, int grid, hipStream_t s);
template <typename T> int batch_blocks_per_cu(int occ);
hipError_t launch_batch_reset(unsigned long long* ticket, int* done, int nseg, int* abort_flag, hipStream_t s);

}  // namespace fockx
