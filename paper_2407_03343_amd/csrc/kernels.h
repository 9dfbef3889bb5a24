// Launchers of the gfx950 kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace smfs {

// Targets per lane of the direct-sum kernels (tiles hold 64 * kDirectTpl).
#ifndef SMFS_DIRECT_TPL
#define SMFS_DIRECT_TPL 2
#endif
constexpr int kDirectTpl = SMFS_DIRECT_TPL;

// Direct sum over target tiles (Section 2.2, eq. uAll) in FP64: every source
// in the given ranges of the packed source array, minus the tile's own
// sphere (the identity self blocks).  Writes per-split partial sums
// part[split][T][3] without the common factor 1/(8 pi mu).
struct DirectArgs {
  const int4 *tiles;        // (first sphere, first target, count, last sphere); NULL: free points
  const int32_t *tsph;      // sphere of every target (tiles that span spheres)
  int64_t n_tiles;
  const double *tgt;        // targets x 3
  int64_t T;                // targets (partial stride)
  const double *src;        // S x 3 positions (packed)
  const double *str;        // S x 3 strengths
  const SphereMeta *meta;
  const SrcRange *ranges;   // source ranges visited
  int32_t n_ranges;
  int64_t range_total;      // sum of range lengths (split base)
  double dscale;            // dipole strengths are multiplied by 2 mu
  int32_t n_splits;
  double *part;
};
hipError_t launch_direct_f64(const DirectArgs &a, hipStream_t s);

// Mixed precision: FP32 sum of the proxy Stokeslets of contact-free
// spheres over the tiles, coordinates relative to sphere centres.
struct Far32Args {
  const int4 *tiles;        // (sphere, first target, count, sphere): one sphere per tile
  int64_t n_tiles;
  const float *tgt32;       // targets minus own centre, T x 3
  const float *src32;       // proxies minus own centre, P*n_proxy x 3 (block 0 order)
  const float *str32;       // proxy strengths (FP32)
  const double *centers;    // P x 3
  const int32_t *free_ids;  // contact-free spheres
  int32_t n_free;
  int32_t n_proxy;
  int32_t n_splits;
  int64_t T;
  float *part32;            // [split][T][3]
};
hipError_t launch_far_f32(const Far32Args &a, hipStream_t s);
// The far-field arguments of a bound problem (api.hip).
Far32Args far32_args(Problem &pb);

// Equivalent-source far field (SMFS_MIXED_EQ): FP32 sum over the
// equivalent Stokeslets of every contact-free sphere that is neither the
// tile's own sphere nor in its near list.
struct EqArgs {
  const int4 *tiles;        // tiles of consecutive targets (may span spheres)
  int64_t n_tiles;
  const int32_t *tsph;      // sphere of each target
  const double *tgt;        // targets, T x 3
  const float *eqpt32;      // equivalent points relative to a centre, n_eq x 3
  const float *q32;         // equivalent strengths, free index major: n_free x n_eq x 3
  const double *centers;    // P x 3
  const int32_t *free_ids;  // free index -> sphere
  const int32_t *near_off;  // P + 1: near list of each target sphere
  const int32_t *near_idx;  // free indices, ascending per sphere
  int32_t n_free, n_eq, n_splits;
  int64_t T;
  float *part32;            // [split][T][3]
};
hipError_t launch_far_eq_f32(const EqArgs &a, hipStream_t s);
// FP64 sum of the proxies of each tile's near contact-free spheres into one
// partial slice (out, T x 3); d supplies targets, sources, strengths, meta.
struct NearArgs {
  DirectArgs d;
  const int4 *tiles;        // one-sphere tiles
  int64_t n_tiles;
  const int32_t *free_ids;
  const int32_t *near_off;
  const int32_t *near_idx;
  double *out;
};
hipError_t launch_near_f64(const NearArgs &a, hipStream_t s);
// q32[q][r] = (float) sum_i E[r + i rows] lambda_hat(proxies of free sphere q)[i]
hipError_t launch_eq_strengths(const double *E, int32_t rows, int32_t cols, const double *lam,
                               const SphereMeta *meta, const int32_t *free_ids, int32_t n_free, float *q32,
                               hipStream_t s);
// Stokeslet matrix without 1/(8 pi mu), 3 nx x 3 ny column-major (set-up)
hipError_t launch_stokeslet_matrix(const double *x, int32_t nx, const double *y, int32_t ny, double *out,
                                   hipStream_t s);
// A[:, c] /= s[c] (column-major, ld rows)
hipError_t launch_scale_cols(double *A, int32_t rows, int32_t cols, const double *sv, hipStream_t s);

// y[i] = base[i] + sw[i/3] * c0 * (sum_s part[s][i] + sum_s part32[s][i])
// (base, sw, part32 nullable)
hipError_t launch_reduce_epilogue(int64_t n3, int32_t n_splits, const double *part, int32_t ns32,
                                  const float *part32, const double *base, const double *sw,
                                  double c0, double *y, hipStream_t s);

// Two-factor pseudo-inverse apply, eq. (transform):
//   s_k = (U_k^T mu_k) / sigma_k      (one wave per task row)
//   lambda_hat[k] = V_k s_k           (scattered to packed source order)
hipError_t launch_pinv_u(const RowTask *tasks, int64_t n, const SphereMeta *meta,
                         const FactorSlot *fs, const double *fac, const double *mu, double *sbuf,
                         hipStream_t s);
// dscale multiplies the dipole strengths (2 mu inside a product with G_hat,
// 1 for physical strengths)
hipError_t launch_pinv_v(const RowTask *tasks, int64_t n, const SphereMeta *meta,
                         const FactorSlot *fs, const double *fac, const double *sbuf,
                         double *lam, double dscale, hipStream_t s);

hipError_t launch_to_f32(int64_t n, const double *x, float *y, hipStream_t s);

// b = W (v + omega x (x - c) - u_inf(x)) per collocation node (bg nullable:
// no background flow; rbm nullable: spheres at rest).
hipError_t launch_rhs(int64_t T, const double *tgt, const int32_t *tsph, const double *sw,
                      const SphereMeta *meta, const double *rbm, double *b, hipStream_t s,
                      const BgFlow *bg = nullptr);
// y = alpha W (v + omega x (x - c) - u_inf(x)) + beta y (y not read when
// beta == 0; bg and rbm nullable as above)
hipError_t launch_rigid(int64_t T, const double *tgt, const int32_t *tsph, const double *sw,
                        const SphereMeta *meta, const double *rbm, double alpha, double beta,
                        double *y, hipStream_t s, const BgFlow *bg = nullptr);
// forces and torques per sphere, F scaled by sF and T by sT
hipError_t launch_force_torque(int32_t P, const SphereMeta *meta, const double *src,
                               const double *lam, double *ft, hipStream_t s, double sF = 1.0,
                               double sT = 1.0);
// y = x with the F rows scaled by sF and the T rows by sT (P x 6)
hipError_t launch_scale_ft(int32_t P, const double *x, double sF, double sT, double *y,
                           hipStream_t s);
// residual statistics: out[0] = max eps_res (masked), out[1] = max |u-ubc|, out[2] = max |ubc|
// with ubc the boundary data of eq. (bc), background flow included (bg nullable)
hipError_t launch_residual_stats(int64_t n, const double *pts, const int32_t *sph,
                                 const SphereMeta *meta, const double *rbm, const double *u,
                                 double floor_rel, double *out, hipStream_t s,
                                 const BgFlow *bg = nullptr);
hipError_t launch_absmax(int64_t n, const double *x, double *out, hipStream_t s);

// Self block B = W G^(kk) of sphere k, column-major rows x cols.
hipError_t launch_assemble_block(const double *tgt, const double *sw, const double *src,
                                 const SphereMeta *meta, int32_t k, int64_t M, int64_t N, double mu,
                                 double *B, hipStream_t s);

// GMRES helpers on a Krylov basis stored as vectors of stride ld.
// beta[0] = ||w|| (and out[0], unless null), then w /= ||w||, or w = 0 when
// ||w|| = 0 (part: nchunks doubles).
hipError_t launch_norm_scale(double *w, int64_t n, double *part, int32_t nchunks, double *beta,
                             double *out, hipStream_t s);
// Delayed classical Gram-Schmidt.  out[0..nv) = V^T a, out[nv..2nv) = V^T b
// over V[0..nv) (part: at least 2 nv nchunks doubles).
hipError_t launch_mdot2(const double *V, int64_t ld, int32_t nv, const double *a, const double *b,
                        int64_t n, double *part, int32_t nchunks, double *out, hipStream_t s);
// From h = [V^T q | V^T w] over V[0..j] (2 (j+1) values): out = [1/nu, gam, nu]
// with nu = sqrt(h_j - sum_{i<j} h_i^2) (1 for j = 0; 0 if not positive)
// and gam = (h_{j+1+j} - sum_{i<j} h_i h_{j+1+i}) / nu.
hipError_t launch_dcgs_coeffs(const double *h, int32_t j, double *out, hipStream_t s);
// q <- (q - V cs) / nu, w <- (w - V cz - q gam) / nu over V[0..nb) with
// coeffs = [1/nu, gam] on the device, then norm[0] = ||w|| and w /= norm[0]
// (part: nparts doubles).
hipError_t launch_dcgs_update(const double *V, int64_t ld, int32_t nb, const double *cs,
                              const double *cz, double *q, double *w, const double *coeffs, int64_t n,
                              double *part, int32_t nparts, double *norm, hipStream_t s);
// y = a*x + b*y ; x,y length n (a, b host scalars)
hipError_t launch_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s);
// y[i] = v
hipError_t launch_fill(int64_t n, double v, double *y, hipStream_t s);
// out = x - y
hipError_t launch_sub(int64_t n, const double *x, const double *y, double *out, hipStream_t s);
// x += sum_j V[j] c[j] (c on device, nv entries)
hipError_t launch_combine(const double *V, int64_t ld, int32_t nv, const double *c, double *x,
                          int64_t n, hipStream_t s);
hipError_t launch_norm2(const double *w, int64_t n, double *part, int32_t nchunks, double *out,
                        hipStream_t s);

int32_t mdot_chunks(int64_t n);

// ---- many right-hand sides ------------------------------------------------
constexpr int kBlockRun = 4;   // right-hand sides sharing one pair geometry

struct BlockDirectArgs {
  const int4 *tiles;        // one-sphere tiles (sphere, first target, count, sphere)
  int64_t n_tiles;
  const double *tgt;
  int64_t T;
  const double *src;
  const double *lamb;       // S x nrhs x 3 (source-major)
  int32_t nrhs;
  const SphereMeta *meta;
  const SrcRange *ranges;
  int32_t n_ranges;
  int64_t range_total;
  int32_t n_splits;
  double *part;             // [split][q][T][3]
};
// Batched pseudo-inverse apply (eq. transform) for nrhs vectors on FP64
// MFMA: S_q = Sigma^-1 U^T mu_q per sphere, then lamb = V S_q scattered to the
// source-major block layout (dipoles times dscale).  Tasks are (sphere,
// first row of a 32-row tile, -, -).
hipError_t launch_pinv_block(const int4 *utasks, int64_t nu, const int4 *vtasks, int64_t nv,
                             const SphereMeta *meta, const FactorSlot *fs, const double *fac,
                             const double *mu, int64_t ldmu, int32_t nrhs, double *S, int64_t lds,
                             double *lamb, double dscale, hipStream_t s);
hipError_t launch_direct_block(const BlockDirectArgs &a, hipStream_t s);
// SMFS_MIXED_EQ for a block of vectors: equivalent strengths of every
// contact-free sphere (q32b [free][n_eq][nrhs][3]), the FP64 near proxies
// into near_out [nrhs][T][3] and the FP32 equivalent-source sum into
// part32b [f.n_splits][nrhs][T][3]; d supplies the one-sphere tiles of
// the near sum, targets, sources and the strengths lamb, f the packed tiles
// of the far sum.
hipError_t launch_eq_block(const BlockDirectArgs &d, const EqArgs &f, const double *E, int32_t n_proxy,
                           float *q32b, double *near_out, float *part32b, hipStream_t s);
hipError_t launch_reduce_block(int64_t n3, int32_t nrhs, int32_t ns, const double *part, int32_t ns32,
                               const float *part32, const double *base, int64_t ldb, const double *sw,
                               double c0, double *y, int64_t ldy, hipStream_t s);
// Mixed precision, many right-hand sides: FP32 far field of the contact-free
// proxies (a.str32 unused; strengths str32b [proxy][nrhs][3], partial sums
// part32b [split][nrhs][T][3], a.n_splits splits over the free spheres).
hipError_t launch_far_block_f32(const Far32Args &a, const float *str32b, int32_t nrhs, float *part32b,
                                hipStream_t s);
hipError_t launch_arnoldi_block(const double *V, int64_t ld, int32_t nrhs, int32_t nv, double *W,
                                int64_t n, double *part, int32_t nchunks, double *h, int32_t ldh,
                                hipStream_t s);
hipError_t launch_norm_scale_block(double *W, int64_t ld, int32_t nrhs, int64_t n, double *part,
                                   int32_t nchunks, double *beta, int32_t ldb, bool scale,
                                   hipStream_t s);
hipError_t launch_scale_block(double *W, int64_t ld, int32_t nrhs, int64_t n, const double *beta,
                              int32_t ldb, hipStream_t s);
hipError_t launch_combine_block(const double *V, int64_t ld, int32_t nrhs, int32_t nv,
                                const double *cf, int32_t ldc, double *X, int64_t ldx, int64_t n,
                                hipStream_t s);

// ---- serving: many independent problems per launch ---------------------
// One entry per resident problem; the product reads x and writes y, the
// Arnoldi pass then orthogonalises y = V + nv ld against V[0..nv).
// One resident request's GMRES cycle on the device (serving): the Arnoldi
// index j within the cycle, the Hessenberg columns in Givens-rotated form,
// the rotations and the rotated right-hand side g.  Every serving kernel
// skips a request whose `active` is 0; k_serve_givens clears it when the
// request needs the host (estimate met, iteration limit, breakdown or the
// end of the cycle).
struct ServeGivens {
  int32_t j, m, active, total, max_it, breakdown;
  double bnorm, tol, est;
  double *H;        // (m + 1) x m, column-major
  double *cs, *sn;  // m each
  double *g;        // m + 1
};

struct ServeDesc {
  DirectArgs da;            // direct sum of this problem (str = lam, own part buffer)
  int64_t tile0;            // first tile of this problem in the launch
  Far32Args fa;             // mixed precision: FP32 far field (n_splits = 0: FP64 product)
  int64_t stile0;           // first one-sphere tile of this problem in the far-field launch
  float *str32;             // FP32 copy of the proxy strengths (the first n_str32 of lam)
  int64_t n_str32;
  const RowTask *utask, *vtask;
  int64_t n_utask, n_vtask, utask0, vtask0;
  const FactorSlot *fs;
  const double *fac;
  double *sbuf;             // Sigma^-1 U^T x per sphere
  double *lam;              // strengths (dipoles times 2 mu), same array as da.str
  const double *sw;         // square-root weights, T
  double c0;                // 1 / (8 pi mu)
  int64_t n;                // 3T
  double *V;                // Krylov basis, stride ld: the product reads V[j], writes V[j + 1]
  int64_t ld;
  ServeGivens *gv;          // the request's cycle state (j, active, ...)
  int32_t nch;              // reduction chunks (mdot_chunks(n))
  double *red;              // reduction partials, at least (j + 1) x nch
  double *h, *h2;           // Gram-Schmidt coefficients of the two passes; h[j + 1] = norm
};
hipError_t launch_serve_product(const ServeDesc *d, int32_t nprob, int64_t tiles, int64_t utasks,
                                int64_t vtasks, int32_t max_splits, int64_t max_n, int64_t stiles,
                                int32_t max_splits32, int64_t max_str32, hipStream_t s);
hipError_t launch_serve_arnoldi(const ServeDesc *d, int32_t nprob, int32_t max_nv, int32_t max_nch,
                                int64_t max_n, hipStream_t s);
// The Givens step of every active request (one thread each): rotates the new
// Hessenberg column h + h2, updates g and j, and clears `active` when the
// request needs the host.
hipError_t launch_serve_givens(const ServeDesc *d, int32_t nprob, hipStream_t s);

// The shared factor 0 applied to all n_free contact-free spheres (their
// sphere ids in free_ids) as two GEMMs on FP64 MFMA; rank and cols are
// factor 0's (host copies, for the grid).  Writes sbuf at each sphere's s0
// and lam at its packed sources, dipoles times dscale.
hipError_t launch_pinv_shared(const int32_t *free_ids, int32_t n_free, int32_t rank, int32_t cols,
                              const SphereMeta *meta, const FactorSlot *fs, const double *fac,
                              const double *mu, double *sbuf, double *lam, double dscale,
                              hipStream_t s);

// FP32 form of launch_pinv_shared for the mixed precision mode, on FP32 MFMA
// with FP32 accumulation: fac32 is the FP32 copy of factor 0 (FP64 offsets
// start at off0), mu is rounded to FP32 as it is read; writes s32 at each
// free sphere's s0 and the FP32 proxy strengths str32 (P*n_proxy x 3).
hipError_t launch_pinv_shared32(const int32_t *free_ids, int32_t n_free, int32_t rank, int32_t cols,
                                const SphereMeta *meta, const FactorSlot *fs, const float *fac32,
                                int64_t off0, const double *mu, float *s32, float *str32,
                                hipStream_t s);

}  // namespace smfs
