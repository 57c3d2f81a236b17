/*
 * fock.h -- C ABI of the exact-exchange (Fock) band-pair path on one MI355X.
 *
 * The operation (Varini et al., "Enhancement of DFT-calculations at
 * Petascale", section 4): for occupied orbitals phi_i with weights f_i and
 * target orbitals psi_j, all given as plane-wave coefficients on one G-sphere,
 *
 *   (V_x psi_j)(G) = - sum_i f_i sum_{G1} c_i(G1) v_ij(G - G1),    G in sphere
 *   v_ij(G)        = K(q+G) rho_ij(G),   K(q+G) = 4 pi / |q+G|^2
 *   rho_ij(G)      = Omega^-1 sum_{G1} conj(c_i(G1)) d_j(G1 + G)
 *
 * i.e. the action of the exchange operator of section 4 (V_x applied to a
 * state, with the overlap charge densities M of the reciprocal-space
 * exchange-energy formula), computed through real space with FFTs as that
 * section describes:  (V_x psi_j) = -(1/(Omega N^2)) sum_i f_i
 * FFT[ phi~_i * BFFT[ K * FFT[ conj(phi~_i) psi~_j ] ] ] on the sphere, with
 * phi~ = BFFT(sphere coefficients), FFT = sum_r e^{-iG.r}, BFFT = sum_G
 * e^{+iG.r}, both unnormalised, N = n1 n2 n3 grid points.
 *
 * Units: Hartree atomic units (bohr, bohr^-1, Hartree).
 * q is the Bloch-vector difference k_target - k_occupied (Cartesian bohr^-1).
 * The single point q + G = 0 (q = 0, G = 0) takes K = 0 (FOCK_G0_ZERO) or the
 * Gygi-Baldereschi constant K0 of the cell's Gamma-centred nq mesh with
 * auxiliary width gb_alpha (FOCK_G0_GB).
 *
 * Memory: orbital coefficients, weights, outputs, workspace and device scalars
 * are DEVICE pointers owned by the caller; fock_cell and its Miller list are
 * HOST memory read during the call only.  Complex data is interleaved
 * (re, im) in the precision the dtype names: complex128 for FOCK_C128 (the
 * FP64 path), complex64 for FOCK_C64 (FP32 transforms and products, FP64
 * energy reduction and G = 0 constant).  Weights and scalars are always FP64.
 * All work is enqueued on `stream` (a hipStream_t; NULL = the null stream);
 * no call synchronises the host.  Calls that share a workspace must not
 * overlap.
 *
 * Errors: arguments are validated on the host before anything is enqueued;
 * on error nothing is written and a status < 0 is returned, with a detail
 * string from fock_last_error() (thread local).  FOCK_E_HIP reports a failed
 * launch; faults of enqueued work surface at the caller's next synchronise.
 */
#ifndef FOCK_H
#define FOCK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FOCK_OK = 0,
  FOCK_E_ARG = -1,              /* null pointer, negative count, ld < npw, bad cell ... */
  FOCK_E_ALIAS = -2,            /* a Miller index |m_a| > (n_a - 1) / 4, or a repeated G */
  FOCK_E_SINGULAR_Q = -3,       /* q != 0 but q + G = 0 for a reciprocal-lattice vector G */
  FOCK_E_WORKSPACE = -4,        /* workspace missing or smaller than fock_workspace_size */
  FOCK_E_UNSUPPORTED_GRID = -5, /* grid shape without compiled transforms */
  FOCK_E_HIP = -6               /* a HIP runtime call failed */
} fock_status;

typedef enum { FOCK_C128 = 0, FOCK_C64 = 1 } fock_dtype;
typedef enum { FOCK_G0_ZERO = 0, FOCK_G0_GB = 1 } fock_g0;

/* The cell, FFT grid and G-sphere (host memory). */
typedef struct {
  double a[3][3];          /* lattice vectors a_1, a_2, a_3 as rows, bohr */
  int32_t n[3];            /* FFT grid n1 x n2 x n3; box is C order, i3 fastest */
  int32_t npw;             /* number of sphere plane waves */
  const int32_t *miller;   /* [npw][3] signed Miller indices; see fock_exchange_grid for the grid rule */
  double ecut_fock;        /* cutoff on |q+G|^2 (bohr^-2) for K; <= 0: whole box */
  int32_t g0;              /* fock_g0 */
  double gb_alpha;         /* FOCK_G0_GB: auxiliary width alpha, bohr^2 (> 0) */
  int32_t nq[3];           /* FOCK_G0_GB: Gamma-centred mesh of the q sum (>= 1) */
} fock_cell;

/* A block of orbitals (device memory). */
typedef struct {
  const void *c;           /* [nb][ld] complex coefficients, in sphere order */
  const double *w;         /* [nb] FP64 occupations (occupied) or weights (targets) */
  int32_t nb;              /* number of orbitals (>= 0) */
  int32_t ld;              /* leading dimension in complex elements (>= npw) */
} fock_orbs;

/* Bytes of device workspace needed by every call below for these sizes. */
size_t fock_workspace_size(const fock_cell *cell, int32_t dtype, int32_t n_occ, int32_t n_tgt);

/* Exchange operator applied to the targets (section 4, V_x on a state):
 * vx_out[j][p] = (V_x psi_j)(G_p), p < npw, device [tgt.nb][tgt.ld]; entries
 * p >= npw are left untouched.  occ.w are the occupations f_i; tgt.w is not
 * read.  The band-pair loop is tiled; the split of the occupied sum into
 * tiles is the band-group split of section 5, summed on the device. */
fock_status fock_apply(const fock_cell *cell, const double q[3], int32_t dtype, const fock_orbs *occ,
                       const fock_orbs *tgt, void *vx_out, void *ws, size_t ws_bytes, void *stream);

/* Allocation-free form of fock_apply, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation): same arguments, result and errors as fock_apply,
 * without the workspace.  The library's per-call device tables (sphere slots,
 * live columns, twiddles) and the fock_apply workspace live in one fixed
 * device array of FOCK_NOALLOC_SCRATCH_BYTES per GPU, part of the library's
 * code object: each GPU the library runs on holds it until the process ends.
 * The call allocates no device memory (its tables reach the device as kernel
 * arguments, stream ordered).  FOCK_E_WORKSPACE when the call would need
 * more than the array (fock_workspace_size plus the tables; e.g. the 24^3
 * grid with 8 occupied and 8 target orbitals fits, a 64^3 grid with 16 does
 * not).  Every call on one GPU uses that GPU's array: calls that overlap in
 * time on one GPU (different streams or threads) race; calls ordered on one
 * stream do not. */
#define FOCK_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
fock_status fock_apply_noalloc(const fock_cell *cell, const double q[3], int32_t dtype, const fock_orbs *occ,
                               const fock_orbs *tgt, void *vx_out, void *stream);

/* Gamma point, real orbitals (section 4 at q = 0, with phi(r) real): V_x of
 * the block applied to itself, vx_out[j][p] = (V_x psi_j)(G_p) with
 * occupations orbs.w, as fock_apply(occ = tgt = orbs, q = 0) returns it.
 * The coefficients must describe real functions: c(-G) = conj(c(G)) on a
 * sphere that holds -G with every G (otherwise the result is undefined).
 * Two real orbitals share one complex transform (psi_2q + i psi_2q+1) and,
 * since K is real and even, each pair transform carries two real pair
 * densities; with the pair symmetry v_ij = v_ji this needs about a quarter of
 * the n_occ x n_tgt pair transforms.  vx_out: device [orbs.nb][orbs.ld].
 * The energy follows as E_x = 1/2 sum_j f_j Re <psi_j | V_x psi_j>. */
size_t fock_workspace_size_gamma(const fock_cell *cell, int32_t dtype, int32_t nb);
fock_status fock_apply_gamma(const fock_cell *cell, int32_t dtype, const fock_orbs *orbs, void *vx_out, void *ws,
                             size_t ws_bytes, void *stream);

/* Exchange energy (section 4, reciprocal-space form):
 * *ex_out = -1/2 sum_ij f_i g_j Omega sum_G K(q+G) |rho_ij(G)|^2, with f = occ.w
 * and g = tgt.w; ex_out is a device FP64 scalar.  Accumulated in FP64 with a
 * fixed reduction order (bitwise reproducible run to run). */
fock_status fock_energy(const fock_cell *cell, const double q[3], int32_t dtype, const fock_orbs *occ,
                        const fock_orbs *tgt, double *ex_out, void *ws, size_t ws_bytes, void *stream);

/* Gradient of fock_energy, scaled by the device FP64 scalar *grad_ex:
 * grad_tgt[j] = grad_ex * dE/d conj(d_j)  =  grad_ex * 1/2 g_j (V_x psi_j)
 * grad_occ[i] = grad_ex * dE/d conj(c_i)  =  grad_ex * 1/2 f_i (V'_x phi_i)
 * (Wirtinger derivatives; V'_x swaps the two blocks and q -> -q).  Either
 * output may be NULL.  Layouts as the inputs ([nb][ld]); only the first npw
 * columns of each row are written.  Pair densities are recomputed, not
 * stored.  With occ and tgt the same block (same c, nb, ld and w) at q = 0
 * the two gradients are equal: one apply fills grad_tgt and is copied. */
fock_status fock_energy_backward(const fock_cell *cell, const double q[3], int32_t dtype, const fock_orbs *occ,
                                 const fock_orbs *tgt, const double *grad_ex, void *grad_occ, void *grad_tgt,
                                 void *ws, size_t ws_bytes, void *stream);

/* Exchange energy over a k-point mesh (section 4: the sums over k and q).
 * sets[k] holds the orbitals at Bloch vector kpts[k] (host [nk][3], bohr^-1),
 * all on the cell's sphere; sets[k].w are the weights (occupation / N_k for a
 * uniform mesh).  Block (k, k') pairs targets at k with occupied orbitals at
 * k', q = k - k' (not folded: the kernel uses |q + G|^2 directly):
 *   E = -1/2 sum_{k,k'} sum_ij w_ik' w_jk Omega sum_G K(k - k' + G) |rho_{ik',jk}(G)|^2.
 * The divergent term (k = k', G = 0) follows cell->g0 (the Gygi-Baldereschi
 * constant of cell->nq, cell->gb_alpha).  Since E_kk' = E_k'k only k <= k' is
 * evaluated.  Device FP64 scalar out.  Workspace: fock_workspace_size_kmesh. */
size_t fock_workspace_size_kmesh(const fock_cell *cell, int32_t dtype, int32_t nk, int32_t nb_max);
fock_status fock_energy_kmesh(const fock_cell *cell, int32_t nk, const double *kpts, int32_t dtype,
                              const fock_orbs *sets, double *ex_out, void *ws, size_t ws_bytes, void *stream);
/* Gradient of fock_energy_kmesh, scaled by the device scalar *grad_ex:
 * grad[k][j] = grad_ex * dE/d conj(c_jk) = grad_ex * w_jk * sum_k' (V_x psi_jk)
 * where V_x uses the occupied set k' and q = k - k'.  grad is a host array of
 * nk device pointers ([nb_k][ld_k] each; a NULL entry skips that set). */
fock_status fock_energy_kmesh_backward(const fock_cell *cell, int32_t nk, const double *kpts, int32_t dtype,
                                       const fock_orbs *sets, const double *grad_ex, void *const *grad, void *ws,
                                       size_t ws_bytes, void *stream);
/* Energy and gradient of fock_energy_kmesh together, from one pass over the
 * pairs: grad[k][j] = dE/d conj(c_jk) (unscaled; every entry of grad with
 * sets[k].nb > 0 must be non-NULL), then *ex_out = 1/2 Re sum_k sum_j
 * sum_p conj(c_jk[p]) grad[k][j][p].  E has degree 2 in the conjugated
 * coefficients, so this equals fock_energy_kmesh up to rounding (the
 * energy pass is not run).  Same workspace as fock_energy_kmesh. */
fock_status fock_energy_kmesh_grad(const fock_cell *cell, int32_t nk, const double *kpts, int32_t dtype,
                                   const fock_orbs *sets, double *ex_out, void *const *grad, void *ws,
                                   size_t ws_bytes, void *stream);

/* Batched form: several independent systems, each an apply as fock_apply
 * (occupied block occ[s], target block tgt[s], q[s]) on its own cell and
 * grid; the band-group sums of section 5 for every system are scheduled
 * together and the whole batch is captured in one hipGraph.  tgt == NULL:
 * every system applies its block to itself; q == NULL: q = 0 for all.
 * Occupied and target coefficients and weights are bound at creation (their
 * contents may change between replays).  The plan owns its device memory,
 * including its results.
 * Two forms of the graph exist and the faster one on this batch is kept:
 *  - every system's own per-shape kernel schedule, one after another;
 *  - when every system is a block applied to itself at q = 0 on a cubic grid
 *    of 24, 48, 64, 72 or 96 points: one persistent kernel for the band-pair
 *    work of all systems (a device work queue of plane, pencil and
 *    multiply-accumulate units with per-segment dependency counters).
 * The choice (and the persistent kernel's pair-tile size, units per work
 * ticket and blocks per compute unit) comes from timing the candidates,
 * unless the JSON tune cache (tune_cache, else $FOCK_TUNE_CACHE; NULL/empty:
 * none) has an entry for the batch signature; the choice is written back.
 * Creation synchronises the device (it runs the candidates). */
fock_status fock_batch_plan_create(const fock_cell *cells, const fock_orbs *occ, const fock_orbs *tgt,
                                   const double (*q)[3], int32_t nsys, int32_t dtype, const char *tune_cache,
                                   void **plan);
/* Replays the graph on the stream, then copies the results out (both stream
 * ordered): vx_out[s] (device [tgt[s].nb][tgt[s].ld], entries p >= npw
 * untouched; vx_out or an entry NULL: not copied) and ex_out[s] = the
 * exchange energy of system s, 1/2 sum_j g_j Re <psi_j | V_x psi_j> with
 * g = tgt[s].w (device FP64 [nsys]; NULL: not copied). */
fock_status fock_batch_apply(void *plan, void *const *vx_out, double *ex_out, void *stream);
/* Synchronises the device and reports a scheduler abort (a dependency wait
 * of the persistent kernel that exceeded its time bound) as FOCK_E_HIP.  The
 * aborted replay's results are undefined; the next replay starts afresh. */
fock_status fock_batch_check(void *plan);
/* Failure detection of the persistent schedule: bound, in milliseconds of
 * the device's constant wall clock, on one dependency wait of a work unit.
 * A wait past it raises the plan's abort flag; every block then stops taking
 * work and the launch drains (no hang), and fock_batch_check reports it.
 * The plan's own bound is 1 s or four times its tuned replay time, whichever
 * is longer (waits in a correct schedule last milliseconds); ms <= 0 restores
 * it.  Takes effect from the next replay; synchronous (a host-to-device copy).
 * Plans without the persistent kernel accept and ignore it. */
fock_status fock_batch_set_wait_limit(void *plan, double ms);
/* JSON description of the chosen schedule (owned by the plan). */
const char *fock_batch_plan_info(void *plan);
void fock_batch_plan_destroy(void *plan);

/* Auxiliary: unnormalised 3-D transform of nb boxes in place (device
 * [nb][n1][n2][n3] complex of dtype); sign = -1 forward (sum e^{-iG.r}),
 * +1 backward.  The same transforms the band-pair path uses; exposed so
 * they can be checked on their own. */
fock_status fock_fft3d(const int32_t n[3], int32_t dtype, int32_t sign, void *x, int32_t nb, void *stream);

/* Band loops of the Car-Parrinello code (section 5: the charge density and
 * the forces on the electronic degrees of freedom are computed band by band,
 * one 3-D FFT per band; the band index is what the band groups split).
 * orbs.c are sphere coefficients of one k-point, orbs.w the occupations f_b;
 * psi_b(r) = Omega^{-1/2} sum_G c_b(G) e^{iG.r} at the grid points
 * r_m = sum_a (m_a / n_a) a_a.  Both calls take the workspace below, any grid
 * that holds the sphere, and run on the stream in order. */
size_t fock_band_workspace_size(const fock_cell *cell, int32_t dtype, int32_t nb);

/* Charge density on the grid: rho_out[m] = sum_b f_b |psi_b(r_m)|^2, device
 * FP64 [n1][n2][n3] (written, not accumulated), for either dtype.  Summed in
 * a fixed order (bitwise reproducible).  cell->ecut_fock is not read. */
fock_status fock_band_density(const fock_cell *cell, int32_t dtype, const fock_orbs *orbs, double *rho_out, void *ws,
                              size_t ws_bytes, void *stream);

/* Force of the local Hamiltonian H = -1/2 nabla^2 + V(r) on each band:
 * force_out[b][p] = -f_b ( 1/2 |k+G_p|^2 c_b(G_p) + (V psi_b)(G_p) ), with
 * (V psi)(G) = N^{-1} sum_m V(r_m) psi~(r_m) e^{-iG.r_m}, psi~ = sum_G c(G) e^{iG.r}
 * (the sphere projection of V psi; -force_out is dE/dconj(c) of
 * E = sum_b f_b <psi_b|H|psi_b>).  vloc: device real potential [n1][n2][n3]
 * in the dtype's precision (double for FOCK_C128, float for FOCK_C64); k: the
 * k-point (host, bohr^-1); force_out: device [orbs.nb][orbs.ld] of dtype,
 * entries p >= npw untouched. */
fock_status fock_band_force(const fock_cell *cell, const double k[3], int32_t dtype, const fock_orbs *orbs,
                            const void *vloc, void *force_out, void *ws, size_t ws_bytes, void *stream);

/* Exchange grid for a reduced Fock cutoff (section 6: the exchange cutoff may
 * be set below the density cutoff, four times the wave-function cutoff).
 * Every call above requires, per axis a, with M_a the largest |m_a| of the
 * sphere and F_a the largest |m_a| of a G with |q+G|^2 <= ecut_fock:
 *     n_a >= min(F_a, 2 M_a) + 2 M_a + 1          (F_a unbounded if ecut_fock <= 0)
 * and returns FOCK_E_ALIAS otherwise.  On such a grid the pair densities are
 * exact wherever K is non-zero and V_x psi is exact on the sphere: the result
 * does not depend on the grid.  F_a is taken as the bound
 * (|a_a| sqrt(ecut_fock) + |a_a . q|) / (2 pi) over the nq vectors q (host,
 * [nq][3]; nq = 0: q = 0).  Writes to n_out the compiled grid of fewest points
 * (for dtype) that meets the rule; cell->n is not read.
 * FOCK_E_UNSUPPORTED_GRID if no compiled grid is large enough. */
fock_status fock_exchange_grid(const fock_cell *cell, int32_t nq, const double *q, int32_t dtype, int32_t n_out[3]);

const char *fock_status_string(fock_status status);
const char *fock_last_error(void);

/* Tracing aid: when enabled, every kernel launch of the calls above is
 * bracketed by HIP events on its stream and attributed to a kernel class
 * (orbital scatter, pair plane FFT, pencil kernel pass, ...).  Returns the
 * number of classes. */
int fock_trace_enable(int on);
/* Accumulated milliseconds and launch counts per class since the last reset
 * (arrays of fock_trace_enable()'s length; either may be NULL).  Waits for the
 * recorded events.  reset != 0 clears the totals. */
int fock_trace_read(double *ms_out, long long *count_out, int reset);
const char *fock_trace_name(int k);

/* Free every cached plan (twiddle tables, sphere index tables) of this process. */
void fock_release_plans(void);

#ifdef __cplusplus
}
#endif

#endif /* FOCK_H */
