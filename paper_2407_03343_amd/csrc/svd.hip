// Truncated SVD of the self blocks B = W G^(kk) on the device (Section 2.2,
// eq. transform; truncation eps_trunc of Section 5), in three stages:
//   B = Q1 R1 and R1^T = Q2 R2 (rocSOLVER geqrf, batched);
//   one-sided Jacobi (Hestenes) on X = R2^T in HIP: X J = U_X Sigma;
//   U = Q1 [U_X; 0] and V = Q2 J (the reflectors of the two QRs applied by
//   k_qr_apply_reg to a whole batch, or by rocSOLVER ormqr per block for
//   blocks of more than 4608 rows), since
//   B = Q1 R2^T Q2^T = Q1 U_X Sigma J^T Q2^T.
// The second QR is a preconditioner: R2^T is much closer to having
// orthogonal columns than R1 (on a 4500 x 1980 contact block the Jacobi
// sweeps drop from over 40 to about 22).
//
// One-sided Jacobi orthogonalises the columns of X by plane rotations,
// each computed from fresh dot products of the two columns it rotates, so
// the singular values come out with the accuracy of the data (the Gram
// matrix is never formed, which would square the condition number and lose
// everything below sqrt(eps) sigma_1, far above the 5e-12 truncation).  The
// columns are processed in blocks of w: a sweep visits every pair of column
// blocks once (round-robin schedule, disjoint pairs in parallel); a pair
// task holds its 2w columns in registers across a 512-thread workgroup (or
// one wave, for blocks of at most 768 columns) and runs one round-robin
// sweep over the 2w columns, accumulating its rotations in a 2w x 2w matrix
// that is applied to V (by a second kernel, or by the one-wave task itself).
// A block whose sweep saw no cosine above its tolerance is left alone by
// the later sweeps.  Sweeps
// repeat until no pair of columns has a cosine above
// max(1e-13, 64 eps ||R||_F / min(|x_a|, |x_b|)): rounding in the rotations
// leaves every column perturbed at the level eps ||R||_F, so a column near
// that level (far below the 5e-12 truncation) has a cosine with any other
// known only to the second bound, and asking for more never ends.  Every
// block is processed on its own, whatever else shares the launch.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <utility>
#include <vector>

#include "../../include/smfs.h"
#include "internal.h"
#include "kernels.h"

namespace smfs {

namespace {

constexpr int kJacThreads = 512;         // threads of a pair task (8 waves)
constexpr int kJacWaves = kJacThreads / 64;
constexpr double kRotTol = 1e-15;        // rotate when |x_a.x_b| > tol |x_a| |x_b|
constexpr double kSweepTol = 1e-13;      // sweeps end when every cosine is below this ...
constexpr double kNoise = 64 * 2.220446049250313e-16;  // ... or below kNoise ||R||_F / min column norm
constexpr int kMaxSweeps = 40;

size_t al256(size_t v) { return (v + 255) / 256 * 256; }

// Round-robin pairing of 2w players: player 0 stays, the others rotate.
__host__ __device__ constexpr int rr_a(int q, int i, int n) { return i == 0 ? 0 : 1 + (q + i) % (n - 1); }
__host__ __device__ constexpr int rr_b(int q, int i, int n) {
  return i == 0 ? 1 + q % (n - 1) : 1 + (q + n - 1 - i) % (n - 1);
}

struct JacArgs {
  double *X;            // per block: n rows x npad columns, column-major (ld n)
  int64_t x_stride;     // elements between blocks
  int32_t n, npad, w;   // rows, padded columns, columns per column block
  const int2 *pairs;    // column-block pairs of this round (npairs), (-1, -1) = none
  int32_t npairs;
  double *Wout;         // per block and pair task: 2w x 2w rotation product (column-major)
  double *off;          // per block and pair task: largest cosine / tolerance seen before rotation
  const double *fro;    // per block: Frobenius norm of R
  const int32_t *skip;  // per block: 1 once its sweeps have converged (its tasks leave it as it is)
  double *V;            // k_jac_pairs_wave: V (npad x npad, column-major per block), updated in the task
  int64_t v_stride;
};

// Shared memory of a pair task.
template <int kW2>
struct JacShared {
  double red[kJacWaves][3 * kW2 / 2];
  double rot[kW2 / 2][2];
  double W[kW2][kW2];
};

// Round q of the inner sweep over the 2w columns held in x (q is a template
// argument so that every column index below is a compile-time constant and
// x stays in registers): dot products of the round's w disjoint pairs,
// reduced over the workgroup, rotations computed by w threads, applied to
// every thread's rows and to W.
template <int kRows, int kW2, int q>
__device__ __forceinline__ void jac_round(double (&x)[kRows][kW2], JacShared<kW2> &sh, double &offmax,
                                          double noise) {
  constexpr int w = kW2 / 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double s[3 * w];
#pragma unroll
  for (int i = 0; i < w; ++i) {
    const int ca = rr_a(q, i, kW2), cb = rr_b(q, i, kW2);
    double aa = 0.0, bb = 0.0, ab = 0.0;
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      aa = fma(x[k][ca], x[k][ca], aa);
      bb = fma(x[k][cb], x[k][cb], bb);
      ab = fma(x[k][ca], x[k][cb], ab);
    }
    s[3 * i] = aa;
    s[3 * i + 1] = bb;
    s[3 * i + 2] = ab;
  }
#pragma unroll
  for (int v = 0; v < 3 * w; ++v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s[v] += __shfl_xor(s[v], o);
  }
  if (lane == 0) {
#pragma unroll
    for (int v = 0; v < 3 * w; ++v) sh.red[wave][v] = s[v];
  }
  __syncthreads();
  if (tid < w) {
    double aa = 0.0, bb = 0.0, ab = 0.0;
    for (int u = 0; u < kJacWaves; ++u) {
      aa += sh.red[u][3 * tid];
      bb += sh.red[u][3 * tid + 1];
      ab += sh.red[u][3 * tid + 2];
    }
    double c = 1.0, sn = 0.0;
    if (aa > 0.0 && bb > 0.0) {
      const double na = sqrt(aa), nb = sqrt(bb);
      const double cosv = fabs(ab) / (na * nb);
      offmax = fmax(offmax, cosv / fmax(kSweepTol, noise / fmin(na, nb)));
      if (cosv > kRotTol) {
        // x_a' = c x_a - s x_b, x_b' = s x_a + c x_b with x_a'.x_b' = 0
        const double zeta = (bb - aa) / (2.0 * ab);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        c = 1.0 / sqrt(1.0 + t * t);
        sn = c * t;
      }
    }
    sh.rot[tid][0] = c;
    sh.rot[tid][1] = sn;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < w; ++i) {
    const int ca = rr_a(q, i, kW2), cb = rr_b(q, i, kW2);
    const double c = sh.rot[i][0], sn = sh.rot[i][1];
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const double xa = x[k][ca], xb = x[k][cb];
      x[k][ca] = c * xa - sn * xb;
      x[k][cb] = sn * xa + c * xb;
    }
  }
  // the same column rotations on W (one row of W per thread)
  if (tid < kW2 * w) {
    const int i = tid / kW2, r = tid % kW2;
    int ca = 0, cb = 0;
#pragma unroll
    for (int ii = 0; ii < w; ++ii)
      if (ii == i) { ca = rr_a(q, ii, kW2); cb = rr_b(q, ii, kW2); }
    const double c = sh.rot[i][0], sn = sh.rot[i][1];
    const double wa = sh.W[r][ca], wb = sh.W[r][cb];
    sh.W[r][ca] = c * wa - sn * wb;
    sh.W[r][cb] = sn * wa + c * wb;
  }
  __syncthreads();
}

template <int kRows, int kW2, int... Q>
__device__ __forceinline__ void jac_rounds(double (&x)[kRows][kW2], JacShared<kW2> &sh, double &offmax,
                                           double noise, std::integer_sequence<int, Q...>) {
  (jac_round<kRows, kW2, Q>(x, sh, offmax, noise), ...);
}

// One pair task: columns of blocks I and J of matrix blockIdx.y.  Each
// thread holds rows tid, tid + 512, ... (kRows of them) of the 2w columns.
template <int kRows, int kW2>
__global__ __launch_bounds__(kJacThreads) void k_jac_pairs(JacArgs a) {
  __shared__ JacShared<kW2> sh;
  const int tid = threadIdx.x;
  const int task = blockIdx.x, b = blockIdx.y;
  const int2 pr = a.pairs[task];
  double *Wo = a.Wout + ((int64_t)b * a.npairs + task) * kW2 * kW2;
  double *offo = a.off + (int64_t)b * a.npairs + task;
  if (pr.x < 0 || a.skip[b]) {
    if (tid == 0) *offo = 0.0;
    return;
  }
  constexpr int w = kW2 / 2;
  double *X = a.X + (int64_t)b * a.x_stride;
  double x[kRows][kW2];
#pragma unroll
  for (int c = 0; c < kW2; ++c) {
    const int64_t gc = c < w ? (int64_t)pr.x * w + c : (int64_t)pr.y * w + (c - w);
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const int r = tid + k * kJacThreads;
      x[k][c] = r < a.n ? X[gc * a.n + r] : 0.0;
    }
  }
  for (int e = tid; e < kW2 * kW2; e += kJacThreads) sh.W[e % kW2][e / kW2] = (e % kW2 == e / kW2) ? 1.0 : 0.0;
  __syncthreads();
  double offmax = 0.0;
  const double noise = kNoise * a.fro[b];
  jac_rounds<kRows, kW2>(x, sh, offmax, noise, std::make_integer_sequence<int, kW2 - 1>{});
#pragma unroll
  for (int c = 0; c < kW2; ++c) {
    const int64_t gc = c < w ? (int64_t)pr.x * w + c : (int64_t)pr.y * w + (c - w);
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const int r = tid + k * kJacThreads;
      if (r < a.n) X[gc * a.n + r] = x[k][c];
    }
  }
  for (int e = tid; e < kW2 * kW2; e += kJacThreads) Wo[e] = sh.W[e % kW2][e / kW2];
  // largest cosine / tolerance of the task (threads < w hold their pairs' maxima)
  if (tid < w) sh.red[0][tid] = offmax;
  __syncthreads();
  if (tid == 0) {
    double m = 0.0;
    for (int i = 0; i < w; ++i) m = fmax(m, sh.red[0][i]);
    *offo = m;
  }
}

// The pair task of k_jac_pairs in one wave, for blocks of at most 64 kRows
// rows: lane l holds rows l, l + 64, ... of the 2w columns and row l of W
// (l < 2w).  The dot products are reduced by an xor butterfly, which leaves
// the same sums, bitwise, in every lane (each step adds the same two
// partials), so every lane computes the same rotations and no barrier is
// needed.  The task then applies W to the 2w columns of V itself (the
// arithmetic of k_jac_vupdate).
template <int kRows, int kW2, int q>
__device__ __forceinline__ void jacw_round(double (&x)[kRows][kW2], double (&wr)[kW2], double &offmax,
                                           double noise) {
  constexpr int w = kW2 / 2;
  double s[3 * w];
#pragma unroll
  for (int i = 0; i < w; ++i) {
    const int ca = rr_a(q, i, kW2), cb = rr_b(q, i, kW2);
    double aa = 0.0, bb = 0.0, ab = 0.0;
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      aa = fma(x[k][ca], x[k][ca], aa);
      bb = fma(x[k][cb], x[k][cb], bb);
      ab = fma(x[k][ca], x[k][cb], ab);
    }
    s[3 * i] = aa;
    s[3 * i + 1] = bb;
    s[3 * i + 2] = ab;
  }
#pragma unroll
  for (int v = 0; v < 3 * w; ++v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s[v] += __shfl_xor(s[v], o);
  }
#pragma unroll
  for (int i = 0; i < w; ++i) {
    const int ca = rr_a(q, i, kW2), cb = rr_b(q, i, kW2);
    const double aa = s[3 * i], bb = s[3 * i + 1], ab = s[3 * i + 2];
    double c = 1.0, sn = 0.0;
    if (aa > 0.0 && bb > 0.0) {
      const double na = sqrt(aa), nb = sqrt(bb);
      const double cosv = fabs(ab) / (na * nb);
      offmax = fmax(offmax, cosv / fmax(kSweepTol, noise / fmin(na, nb)));
      if (cosv > kRotTol) {
        // x_a' = c x_a - s x_b, x_b' = s x_a + c x_b with x_a'.x_b' = 0
        const double zeta = (bb - aa) / (2.0 * ab);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        c = 1.0 / sqrt(1.0 + t * t);
        sn = c * t;
      }
    }
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const double xa = x[k][ca], xb = x[k][cb];
      x[k][ca] = c * xa - sn * xb;
      x[k][cb] = sn * xa + c * xb;
    }
    const double wa = wr[ca], wb = wr[cb];
    wr[ca] = c * wa - sn * wb;
    wr[cb] = sn * wa + c * wb;
  }
}

template <int kRows, int kW2, int... Q>
__device__ __forceinline__ void jacw_rounds(double (&x)[kRows][kW2], double (&wr)[kW2], double &offmax,
                                            double noise, std::integer_sequence<int, Q...>) {
  (jacw_round<kRows, kW2, Q>(x, wr, offmax, noise), ...);
}

template <int kRows, int kW2>
__device__ __forceinline__ void jac_pair_wave(const JacArgs &a) {
  const int lane = threadIdx.x;
  const int task = blockIdx.x, b = blockIdx.y;
  const int2 pr = a.pairs[task];
  double *offo = a.off + (int64_t)b * a.npairs + task;
  if (pr.x < 0 || a.skip[b]) {
    if (lane == 0) *offo = 0.0;
    return;
  }
  constexpr int w = kW2 / 2;
  double *X = a.X + (int64_t)b * a.x_stride;
  double x[kRows][kW2];
#pragma unroll
  for (int c = 0; c < kW2; ++c) {
    const int64_t gc = c < w ? (int64_t)pr.x * w + c : (int64_t)pr.y * w + (c - w);
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const int r = lane + 64 * k;
      x[k][c] = r < a.n ? X[gc * a.n + r] : 0.0;
    }
  }
  double wr[kW2];
#pragma unroll
  for (int c = 0; c < kW2; ++c) wr[c] = c == lane ? 1.0 : 0.0;
  double offmax = 0.0;
  jacw_rounds<kRows, kW2>(x, wr, offmax, kNoise * a.fro[b], std::make_integer_sequence<int, kW2 - 1>{});
#pragma unroll
  for (int c = 0; c < kW2; ++c) {
    const int64_t gc = c < w ? (int64_t)pr.x * w + c : (int64_t)pr.y * w + (c - w);
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const int r = lane + 64 * k;
      if (r < a.n) X[gc * a.n + r] = x[k][c];
    }
  }
  // V[:, I u J] <- V[:, I u J] W, W through LDS into every lane's registers
  __shared__ double Ws[kW2 * kW2];
  if (lane < kW2) {
#pragma unroll
    for (int c = 0; c < kW2; ++c) Ws[c * kW2 + lane] = wr[c];
  }
  __syncthreads();
  double W[kW2 * kW2];
#pragma unroll
  for (int e = 0; e < kW2 * kW2; ++e) W[e] = Ws[e];
  // V is column-major here: the lanes read consecutive rows of a column
  double *Vb = a.V + (int64_t)b * a.v_stride;
  double *vc[kW2];
#pragma unroll
  for (int c = 0; c < kW2; ++c)
    vc[c] = Vb + (c < w ? (int64_t)pr.x * w + c : (int64_t)pr.y * w + (c - w)) * a.npad;
  for (int r = lane; r < a.npad; r += 64) {
    double v[kW2];
#pragma unroll
    for (int c = 0; c < kW2; ++c) v[c] = vc[c][r];
#pragma unroll
    for (int c = 0; c < kW2; ++c) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < kW2; ++k) t = fma(v[k], W[c * kW2 + k], t);
      vc[c][r] = t;
    }
  }
  if (lane == 0) *offo = offmax;
}

// Blocks of at most 512 rows: two waves per SIMD (the register budget of
// 256 still holds the task); 768 rows need more registers than that.
template <int kRows, int kW2>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_jac_pairs_wave(JacArgs a) {
  jac_pair_wave<kRows, kW2>(a);
}
template <int kRows, int kW2>
__global__ __launch_bounds__(64) void k_jac_pairs_wave_wide(JacArgs a) {
  jac_pair_wave<kRows, kW2>(a);
}

// V (npad x npad, row-major per block) <- V[:, I u J] W for every pair task
// of the round: one thread per row.
template <int kW2>
__global__ __launch_bounds__(256) void k_jac_vupdate(double *V, int64_t v_stride, int32_t npad,
                                                     const int2 *pairs, int32_t npairs, const double *Wbuf,
                                                     const int32_t *skip) {
  __shared__ double W[kW2 * kW2];
  const int task = blockIdx.y, b = blockIdx.z;
  const int2 pr = pairs[task];
  if (pr.x < 0 || skip[b]) return;
  const double *Wi = Wbuf + ((int64_t)b * npairs + task) * kW2 * kW2;
  for (int e = threadIdx.x; e < kW2 * kW2; e += blockDim.x) W[e] = Wi[e];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= npad) return;
  constexpr int w = kW2 / 2;
  double *row = V + (int64_t)b * v_stride + r * npad;
  double v[kW2];
#pragma unroll
  for (int c = 0; c < w; ++c) {
    v[c] = row[(int64_t)pr.x * w + c];
    v[w + c] = row[(int64_t)pr.y * w + c];
  }
#pragma unroll
  for (int c = 0; c < kW2; ++c) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kW2; ++k) s = fma(v[k], W[c * kW2 + k], s);
    if (c < w) row[(int64_t)pr.x * w + c] = s;
    else row[(int64_t)pr.y * w + (c - w)] = s;
  }
}

// C <- Q C for the Householder QR of every block of a batch (the geqrf
// layout: reflector k is column k of A below the diagonal with an implicit
// 1 on it; Q = H_0 H_1 ... H_{K-1}, H_k = I - tau_k v_k v_k^T), the
// reflectors applied last to first.  One wave per block (blockIdx.y) and kC
// columns of C (blockIdx.x), held in registers for the whole sweep over the
// reflectors (blocks of at most 64 kR rows): lane l holds rows l, l + 64,
// ... of the kC columns, and only the reflectors are read per step.  Block
// b's C has ncols[b] columns of leading dimension ldc, at Cp[b] (or at
// Cbase + b c_stride when Cp is null).
template <int kR, int kC>
__global__ __launch_bounds__(64) void k_qr_apply_reg(const double *A, int64_t a_stride, int32_t m, int32_t K,
                                                     const double *tau, int64_t tau_stride, double *const *Cp,
                                                     double *Cbase, int64_t c_stride, int32_t ldc,
                                                     const int32_t *ncols) {
  const int b = blockIdx.y, lane = threadIdx.x;
  const int c0 = blockIdx.x * kC;
  const int nc = ncols[b];
  if (c0 >= nc) return;
  const int cn = min(kC, nc - c0);
  const double *Ab = A + (int64_t)b * a_stride;
  double *C = (Cp ? Cp[b] : Cbase + (int64_t)b * c_stride) + (int64_t)c0 * ldc;
  double c[kR][kC];
#pragma unroll
  for (int t = 0; t < kR; ++t) {
    const int i = lane + 64 * t;
#pragma unroll
    for (int j = 0; j < kC; ++j) c[t][j] = (i < m && j < cn) ? C[(int64_t)j * ldc + i] : 0.0;
  }
  for (int k = K - 1; k >= 0; --k) {
    const double tk = tau[(int64_t)b * tau_stride + k];
    if (tk == 0.0) continue;
    const double *v = Ab + (int64_t)k * m;
    double vv[kR], w[kC];
#pragma unroll
    for (int j = 0; j < kC; ++j) w[j] = 0.0;
#pragma unroll
    for (int t = 0; t < kR; ++t) {
      const int i = lane + 64 * t;
      vv[t] = i == k ? 1.0 : (i > k && i < m ? v[i] : 0.0);
#pragma unroll
      for (int j = 0; j < kC; ++j) w[j] = fma(vv[t], c[t][j], w[j]);
    }
#pragma unroll
    for (int j = 0; j < kC; ++j) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) w[j] += __shfl_xor(w[j], o);
      w[j] *= -tk;
    }
#pragma unroll
    for (int t = 0; t < kR; ++t) {
#pragma unroll
      for (int j = 0; j < kC; ++j) c[t][j] = fma(w[j], vv[t], c[t][j]);
    }
  }
#pragma unroll
  for (int t = 0; t < kR; ++t) {
    const int i = lane + 64 * t;
    if (i < m) {
#pragma unroll
      for (int j = 0; j < kC; ++j)
        if (j < cn) C[(int64_t)j * ldc + i] = c[t][j];
    }
  }
}

// C <- Q C for every block of a batch (k_qr_apply_reg), for blocks of at
// most 4608 rows.
hipError_t launch_qr_apply(const double *A, int64_t a_stride, int32_t m, int32_t K, const double *tau,
                           int64_t tau_stride, double *const *Cp, double *Cbase, int64_t c_stride, int32_t ldc,
                           const int32_t *ncols, int32_t max_cols, int32_t nb, hipStream_t s) {
  auto grid = [&](int kc) { return dim3((unsigned)((max_cols + kc - 1) / kc), (unsigned)nb); };
  if (m <= 512)
    hipLaunchKernelGGL((k_qr_apply_reg<8, 8>), grid(8), dim3(64), 0, s, A, a_stride, m, K, tau, tau_stride, Cp,
                       Cbase, c_stride, ldc, ncols);
  else if (m <= 1024)
    hipLaunchKernelGGL((k_qr_apply_reg<16, 4>), grid(4), dim3(64), 0, s, A, a_stride, m, K, tau, tau_stride, Cp,
                       Cbase, c_stride, ldc, ncols);
  else if (m <= 1536)
    hipLaunchKernelGGL((k_qr_apply_reg<24, 2>), grid(2), dim3(64), 0, s, A, a_stride, m, K, tau, tau_stride, Cp,
                       Cbase, c_stride, ldc, ncols);
  else if (m <= 2048)
    hipLaunchKernelGGL((k_qr_apply_reg<32, 2>), grid(2), dim3(64), 0, s, A, a_stride, m, K, tau, tau_stride, Cp,
                       Cbase, c_stride, ldc, ncols);
  else if (m <= 3072)
    hipLaunchKernelGGL((k_qr_apply_reg<48, 1>), grid(1), dim3(64), 0, s, A, a_stride, m, K, tau, tau_stride, Cp,
                       Cbase, c_stride, ldc, ncols);
  else
    hipLaunchKernelGGL((k_qr_apply_reg<72, 1>), grid(1), dim3(64), 0, s, A, a_stride, m, K, tau, tau_stride, Cp,
                       Cbase, c_stride, ldc, ncols);
  return hipGetLastError();
}

// T = R1^T (n x n, column-major, lower triangular) from the upper triangle
// of the first QR (m x n, column-major, ld m).
__global__ void k_jac_transpose(const double *A, int64_t a_stride, int32_t m, int32_t n, double *T,
                                int64_t t_stride) {
  const int b = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int64_t r = idx % n, c = idx / n;   // T(r, c) = R1(c, r)
  T[(int64_t)b * t_stride + idx] = r >= c ? A[(int64_t)b * a_stride + r * m + c] : 0.0;
}

// X = R2^T (n rows, npad columns, column-major; zero above the diagonal and
// in padded columns) from the upper triangle of the second QR (n x n, ld n),
// V = I.
__global__ void k_jac_init(const double *T, int64_t t_stride, int32_t n, double *X, int64_t x_stride,
                           int32_t npad, double *V, int64_t v_stride) {
  const int b = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (int64_t)n * npad) {
    const int64_t r = idx % n, c = idx / n;   // X(r, c) = R2(c, r)
    X[(int64_t)b * x_stride + idx] = (c < n && r >= c) ? T[(int64_t)b * t_stride + r * n + c] : 0.0;
  }
  if (idx < (int64_t)npad * npad) {
    const int64_t r = idx / npad, c = idx % npad;
    V[(int64_t)b * v_stride + idx] = r == c ? 1.0 : 0.0;
  }
}

// Column norms of X: one wave per column.
__global__ __launch_bounds__(256) void k_jac_colnorm(const double *X, int64_t x_stride, int32_t n, int32_t npad,
                                                     double *sig) {
  const int b = blockIdx.y;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (c >= npad) return;
  const double *col = X + (int64_t)b * x_stride + (int64_t)c * n;
  double s = 0.0;
  for (int r = lane; r < n; r += 64) s = fma(col[r], col[r], s);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) sig[(int64_t)b * npad + c] = sqrt(s);
}

// Frobenius norm of each block's X (= R): one workgroup per block.
__global__ __launch_bounds__(1024) void k_jac_fro(const double *X, int64_t x_stride, int64_t count, double *fro) {
  __shared__ double red[16];
  const int b = blockIdx.x;
  const double *xb = X + (int64_t)b * x_stride;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += blockDim.x) s = fma(xb[i], xb[i], s);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int u = 0; u < (int)(blockDim.x >> 6); ++u) t += red[u];
    fro[b] = sqrt(t);
  }
}

struct FinalArgs {
  const double *X;
  int64_t x_stride;
  const double *V;
  int64_t v_stride;
  const double *sig;       // unsorted column norms, npad per block
  const int32_t *perm;     // per block: n source columns in descending order of norm
  const int32_t *rank;     // per block
  int32_t m, n, npad;
  int32_t v_colmajor;      // V column-major (the one-wave pair tasks) rather than row-major
  double *const *U;        // per block: slot U (m x n, column-major), V (n x n row-major), sigma
  double *const *Vs;
  double *const *Ss;
};

// Slot outputs of block blockIdx.y, column c = blockIdx.x, with j =
// perm[c]: U[:, c] = [x_j / sigma_j; 0], sigma[c] = sigma_j; columns at or
// beyond the rank are left alone.
__global__ __launch_bounds__(256) void k_jac_finalize_u(FinalArgs f) {
  const int b = blockIdx.y, c = blockIdx.x;
  if (c >= f.rank[b]) return;
  const int j = f.perm[(int64_t)b * f.n + c];
  const double s = f.sig[(int64_t)b * f.npad + j];
  const double inv = 1.0 / s;
  const double *xc = f.X + (int64_t)b * f.x_stride + (int64_t)j * f.n;
  double *u = f.U[b] + (int64_t)c * f.m;
  for (int r = threadIdx.x; r < f.m; r += blockDim.x) u[r] = r < f.n ? xc[r] * inv : 0.0;
  if (threadIdx.x == 0) f.Ss[b][c] = s;
}

// Jp[:, c] = J[:, perm[c]] (n x rank, column-major, ld n, written over X
// once U is out), the rotations in the kept order.
__global__ __launch_bounds__(256) void k_jac_finalize_j(FinalArgs f, double *Jp) {
  const int b = blockIdx.y, c = blockIdx.x;
  if (c >= f.rank[b]) return;
  const int j = f.perm[(int64_t)b * f.n + c];
  const double *vb = f.V + (int64_t)b * f.v_stride;
  double *jc = Jp + (int64_t)b * f.x_stride + (int64_t)c * f.n;
  for (int r = threadIdx.x; r < f.n; r += blockDim.x)
    jc[r] = f.v_colmajor ? vb[(int64_t)j * f.npad + r] : vb[(int64_t)r * f.npad + j];
}

// Slot V (n x n row-major, rank columns) from Q2 Jp (n x rank, column-major).
__global__ __launch_bounds__(256) void k_jac_store_v(FinalArgs f, const double *QJ) {
  const int b = blockIdx.y, c = blockIdx.x;
  if (c >= f.rank[b]) return;
  const double *qc = QJ + (int64_t)b * f.x_stride + (int64_t)c * f.n;
  double *vs = f.Vs[b];
  for (int r = threadIdx.x; r < f.n; r += blockDim.x) vs[(int64_t)r * f.n + c] = qc[r];
}

// Round-robin schedule of nbk (even) column blocks: round r pairs.
std::vector<int2> block_schedule(int nbk) {
  std::vector<int2> out;
  for (int q = 0; q < nbk - 1; ++q)
    for (int i = 0; i < nbk / 2; ++i) out.push_back(make_int2(rr_a(q, i, nbk), rr_b(q, i, nbk)));
  return out;
}

}  // namespace

// Column-block width and rows per thread for n rows: the 2w columns of a
// pair task must fit in registers, across one wave (n <= 768) or across 512
// threads.
int jacobi_shape(int n, int &w, int &rows, bool &wave) {
  wave = n <= 768;   // one wave per pair task, 4 / 8 / 12 rows per lane
  if (wave) { w = 4; rows = n <= 256 ? 4 : n <= 512 ? 8 : 12; return SMFS_OK; }
  if (n <= 2048) { w = 8; rows = 4; return SMFS_OK; }
  if (n <= 4096) { w = 4; rows = 8; return SMFS_OK; }
  set_error("device SVD: blocks with more than 4096 columns are not supported");
  return SMFS_E_UNSUPPORTED;
}

// Scratch of one batch of nb blocks of shape m x n (JacPlan): rocSOLVER's
// work arrays (geqrf, ormqr), the blocks and their QR scalars, R1^T and its
// QR scalars, X, V, rotation products, cosines, norms, permutations, ranks,
// slot pointers, schedule.
int jacobi_plan(rocblas_handle h, int m, int n, int nb, JacPlan &p) {
  int rc = jacobi_shape(n, p.w, p.rows, p.wave);
  if (rc) return rc;
  p.npad = (n + p.w - 1) / p.w * p.w;
  p.nbk = p.npad / p.w;
  if (p.nbk % 2) { p.nbk += 1; p.npad += p.w; }
  p.npairs = p.nbk / 2;
  double *fake = reinterpret_cast<double *>((uintptr_t)4096);
  size_t w1 = 0, w2 = 0, w3 = 0, w4 = 0;
  rocblas_start_device_memory_size_query(h);
  rocblas_status q1 = rocsolver_dgeqrf_strided_batched(h, m, n, fake, m, (rocblas_stride)m * n, fake, n, nb);
  rocblas_stop_device_memory_size_query(h, &w1);
  rocblas_start_device_memory_size_query(h);
  rocblas_status q2 = rocsolver_dormqr(h, rocblas_side_left, rocblas_operation_none, m, n, n, fake, m, fake,
                                       fake, m);
  rocblas_stop_device_memory_size_query(h, &w2);
  rocblas_start_device_memory_size_query(h);
  rocblas_status q3 = rocsolver_dgeqrf_strided_batched(h, n, n, fake, n, (rocblas_stride)n * n, fake, n, nb);
  rocblas_stop_device_memory_size_query(h, &w3);
  rocblas_start_device_memory_size_query(h);
  rocblas_status q4 = rocsolver_dormqr(h, rocblas_side_left, rocblas_operation_none, n, n, n, fake, n, fake,
                                       fake, n);
  rocblas_stop_device_memory_size_query(h, &w4);
  auto ok = [](rocblas_status q) {
    return q == rocblas_status_success || q == rocblas_status_size_increased || q == rocblas_status_size_unchanged;
  };
  if (!ok(q1) || !ok(q2) || !ok(q3) || !ok(q4)) {
    set_error("device SVD: workspace query failed");
    return SMFS_E_SVD;
  }
  p.work = al256(std::max(std::max(w1, w2), std::max(w3, w4)));
  p.a = al256(sizeof(double) * (size_t)m * n * nb);
  p.tau = al256(sizeof(double) * (size_t)n * nb);
  p.t = al256(sizeof(double) * (size_t)n * n * nb);
  p.tau2 = al256(sizeof(double) * (size_t)n * nb);
  p.x = al256(sizeof(double) * (size_t)n * p.npad * nb);
  p.v = al256(sizeof(double) * (size_t)p.npad * p.npad * nb);
  p.wbuf = al256(sizeof(double) * (size_t)nb * p.npairs * 4 * p.w * p.w);
  p.off = al256(sizeof(double) * (size_t)nb * p.npairs * (p.nbk - 1));
  p.sig = al256(sizeof(double) * (size_t)nb * p.npad);
  p.fro = al256(sizeof(double) * (size_t)nb);
  p.perm = al256(sizeof(int32_t) * (size_t)nb * n);
  p.rank = al256(sizeof(int32_t) * (size_t)nb);
  p.ptrs = al256(sizeof(double *) * 3 * (size_t)nb);
  p.sched = al256(sizeof(int2) * (size_t)(p.nbk - 1) * p.npairs);
  p.skip = al256(sizeof(int32_t) * (size_t)nb);
  p.total = p.work + p.a + p.tau + p.t + p.tau2 + p.x + p.v + p.wbuf + p.off + p.sig + p.fro + p.perm + p.rank +
            p.ptrs + p.sched + p.skip;
  return SMFS_OK;
}

// Factor nb blocks of shape m x n already assembled at the plan's A region
// of scratch: slots get U (m x rank), V (n x n row-major, rank columns) and
// sigma (descending), ranks[q] the kept count (sigma > trunc sigma_1).
int jacobi_svd_batch(rocblas_handle h, const JacPlan &p, char *scratch, int m, int n, int nb,
                     double *const *U, double *const *Vs, double *const *Ss, double trunc, int *ranks,
                     int *sweeps_out, hipStream_t s) {
  char *o = scratch;
  char *work = o; o += p.work;
  double *A = (double *)o; o += p.a;
  double *tau = (double *)o; o += p.tau;
  double *T = (double *)o; o += p.t;
  double *tau2 = (double *)o; o += p.tau2;
  double *X = (double *)o; o += p.x;
  double *V = (double *)o; o += p.v;
  double *Wb = (double *)o; o += p.wbuf;
  double *off = (double *)o; o += p.off;
  double *sig = (double *)o; o += p.sig;
  double *fro = (double *)o; o += p.fro;
  int32_t *perm = (int32_t *)o; o += p.perm;
  int32_t *drank = (int32_t *)o; o += p.rank;
  double **ptrs = (double **)o; o += p.ptrs;
  int2 *sched = (int2 *)o; o += p.sched;
  int32_t *skip = (int32_t *)o; o += p.skip;
  if (rocblas_set_workspace(h, work, p.work) != rocblas_status_success) {
    set_error("device SVD: rocblas_set_workspace failed");
    return SMFS_E_DEVICE;
  }
  struct Reset {
    rocblas_handle h;
    ~Reset() { (void)rocblas_set_workspace(h, nullptr, 0); }
  } reset{h};
  // B = Q1 R1 for every block, then R1^T = Q2 R2
  if (rocsolver_dgeqrf_strided_batched(h, m, n, A, m, (rocblas_stride)m * n, tau, n, nb) != rocblas_status_success) {
    set_error("device SVD: geqrf failed");
    return SMFS_E_SVD;
  }
  const int64_t ts = (int64_t)n * n;
  hipLaunchKernelGGL(k_jac_transpose, dim3((unsigned)((ts + 255) / 256), nb), dim3(256), 0, s, A, (int64_t)m * n, m,
                     n, T, ts);
  SMFS_HIP(hipGetLastError());
  if (rocsolver_dgeqrf_strided_batched(h, n, n, T, n, (rocblas_stride)ts, tau2, n, nb) != rocblas_status_success) {
    set_error("device SVD: geqrf of R^T failed");
    return SMFS_E_SVD;
  }
  const int64_t xs = (int64_t)n * p.npad, vs = (int64_t)p.npad * p.npad;
  {
    const int64_t cnt = std::max<int64_t>((int64_t)n * p.npad, vs);
    hipLaunchKernelGGL(k_jac_init, dim3((unsigned)((cnt + 255) / 256), nb), dim3(256), 0, s, T, ts, n, X, xs,
                       p.npad, V, vs);
    SMFS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_jac_fro, dim3(nb), dim3(1024), 0, s, X, xs, xs, fro);
    SMFS_HIP(hipGetLastError());
  }
  const std::vector<int2> sch = block_schedule(p.nbk);
  std::vector<int2> sch_host(sch);
  // the padded block (index nbk - 1 when n's blocks are odd) pairs with a
  // real block: both stay as they are (zero columns do not rotate), so the
  // task runs normally
  SMFS_HIP(hipMemcpyAsync(sched, sch_host.data(), sizeof(int2) * sch_host.size(), hipMemcpyHostToDevice, s));
  const int rounds = p.nbk - 1;
  std::vector<double> offh((size_t)nb * p.npairs * rounds);
  // a block whose sweep saw no cosine above its tolerance is left alone by
  // the later sweeps, so that its factors do not depend on the other blocks
  // of the batch
  std::vector<int32_t> skiph(nb, 0);
  SMFS_HIP(hipMemcpyAsync(skip, skiph.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, s));
  int sweep = 0;
  for (; sweep < kMaxSweeps; ++sweep) {
    for (int r = 0; r < rounds; ++r) {
      JacArgs ja;
      ja.X = X;
      ja.x_stride = xs;
      ja.n = n;
      ja.npad = p.npad;
      ja.w = p.w;
      ja.pairs = sched + (int64_t)r * p.npairs;
      ja.npairs = p.npairs;
      ja.Wout = Wb;
      ja.off = off + (int64_t)r * nb * p.npairs;
      ja.fro = fro;
      ja.skip = skip;
      ja.V = V;
      ja.v_stride = vs;
      const dim3 g((unsigned)p.npairs, (unsigned)nb);
      if (p.wave && p.rows == 4) hipLaunchKernelGGL((k_jac_pairs_wave<4, 8>), g, dim3(64), 0, s, ja);
      else if (p.wave && p.rows == 8) hipLaunchKernelGGL((k_jac_pairs_wave<8, 8>), g, dim3(64), 0, s, ja);
      else if (p.wave) hipLaunchKernelGGL((k_jac_pairs_wave_wide<12, 8>), g, dim3(64), 0, s, ja);
      else if (p.w == 8) hipLaunchKernelGGL((k_jac_pairs<4, 16>), g, dim3(kJacThreads), 0, s, ja);
      else hipLaunchKernelGGL((k_jac_pairs<8, 8>), g, dim3(kJacThreads), 0, s, ja);
      SMFS_HIP(hipGetLastError());
      if (p.wave) continue;   // the one-wave tasks update V themselves
      const dim3 gv((unsigned)((p.npad + 255) / 256), (unsigned)p.npairs, (unsigned)nb);
      if (p.w == 8)
        hipLaunchKernelGGL((k_jac_vupdate<16>), gv, dim3(256), 0, s, V, vs, p.npad, ja.pairs, p.npairs, Wb, skip);
      else
        hipLaunchKernelGGL((k_jac_vupdate<8>), gv, dim3(256), 0, s, V, vs, p.npad, ja.pairs, p.npairs, Wb, skip);
      SMFS_HIP(hipGetLastError());
    }
    SMFS_HIP(hipMemcpyAsync(offh.data(), off, sizeof(double) * offh.size(), hipMemcpyDeviceToHost, s));
    SMFS_HIP(hipStreamSynchronize(s));
    // offh: [round][block][task]
    bool all = true;
    for (int b = 0; b < nb; ++b) {
      if (skiph[b]) continue;
      double mx = 0.0;
      for (int r = 0; r < rounds; ++r)
        for (int t = 0; t < p.npairs; ++t) mx = std::max(mx, offh[((size_t)r * nb + b) * p.npairs + t]);
      if (!(mx >= 0.0)) {
        set_error("device SVD: non-finite rotation");
        return SMFS_E_SVD;
      }
      if (mx < 1.0) skiph[b] = 1;
      else all = false;
    }
    if (all) { ++sweep; break; }
    SMFS_HIP(hipMemcpyAsync(skip, skiph.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, s));
  }
  if (sweeps_out) *sweeps_out = sweep;
  if (sweep >= kMaxSweeps) {
    set_error("device SVD: Jacobi sweeps did not converge");
    return SMFS_E_SVD;
  }
  // singular values: column norms, sorted on the host
  hipLaunchKernelGGL(k_jac_colnorm, dim3((unsigned)((p.npad + 3) / 4), nb), dim3(256), 0, s, X, xs, n, p.npad, sig);
  SMFS_HIP(hipGetLastError());
  std::vector<double> sh((size_t)nb * p.npad);
  SMFS_HIP(hipMemcpyAsync(sh.data(), sig, sizeof(double) * sh.size(), hipMemcpyDeviceToHost, s));
  SMFS_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> ph((size_t)nb * n), rh(nb);
  for (int q = 0; q < nb; ++q) {
    const double *sq = sh.data() + (size_t)q * p.npad;
    int32_t *pq = ph.data() + (size_t)q * n;
    std::iota(pq, pq + n, 0);
    std::stable_sort(pq, pq + n, [sq](int32_t x, int32_t y) { return sq[x] > sq[y]; });
    const double s1 = sq[pq[0]];
    if (!(s1 > 0.0) || !std::isfinite(s1)) {
      set_error("device SVD: zero or non-finite block");
      return SMFS_E_SVD;
    }
    int r = 0;
    while (r < n && sq[pq[r]] > trunc * s1) ++r;
    rh[q] = r;
    ranks[q] = r;
  }
  std::vector<double *> hp(3 * (size_t)nb);
  for (int q = 0; q < nb; ++q) {
    hp[q] = U[q];
    hp[nb + q] = Vs[q];
    hp[2 * nb + q] = Ss[q];
  }
  SMFS_HIP(hipMemcpyAsync(perm, ph.data(), sizeof(int32_t) * ph.size(), hipMemcpyHostToDevice, s));
  SMFS_HIP(hipMemcpyAsync(drank, rh.data(), sizeof(int32_t) * rh.size(), hipMemcpyHostToDevice, s));
  SMFS_HIP(hipMemcpyAsync(ptrs, hp.data(), sizeof(double *) * hp.size(), hipMemcpyHostToDevice, s));
  FinalArgs f;
  f.X = X;
  f.x_stride = xs;
  f.V = V;
  f.v_stride = vs;
  f.sig = sig;
  f.perm = perm;
  f.rank = drank;
  f.m = m;
  f.n = n;
  f.npad = p.npad;
  f.v_colmajor = p.wave ? 1 : 0;
  f.U = ptrs;
  f.Vs = ptrs + nb;
  f.Ss = ptrs + 2 * nb;
  hipLaunchKernelGGL(k_jac_finalize_u, dim3((unsigned)n, nb), dim3(256), 0, s, f);
  SMFS_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_jac_finalize_j, dim3((unsigned)n, nb), dim3(256), 0, s, f, X);
  SMFS_HIP(hipGetLastError());
  // U = Q1 [U_X; 0] and V = Q2 J with the reflectors of the two QRs: one
  // launch for the whole batch when the columns fit in registers (at most
  // 4608 rows), else one rocSOLVER ormqr per block.  The choice depends on
  // the block's shape only, so a block's factors do not depend on its batch.
  const int rmax = *std::max_element(rh.begin(), rh.end());
  if (m <= 4608) {
    SMFS_HIP(launch_qr_apply(A, (int64_t)m * n, m, n, tau, (int64_t)n, ptrs, nullptr, 0, m, drank, rmax, nb, s));
  } else {
    for (int q = 0; q < nb; ++q)
      if (rocsolver_dormqr(h, rocblas_side_left, rocblas_operation_none, m, rh[q], n, A + (size_t)q * m * n, m,
                           tau + (size_t)q * n, U[q], m) != rocblas_status_success) {
        set_error("device SVD: ormqr failed");
        return SMFS_E_SVD;
      }
  }
  // n <= 4096 (jacobi_shape)
  SMFS_HIP(launch_qr_apply(T, ts, n, n, tau2, (int64_t)n, nullptr, X, xs, n, drank, rmax, nb, s));
  hipLaunchKernelGGL(k_jac_store_v, dim3((unsigned)n, nb), dim3(256), 0, s, f, X);
  SMFS_HIP(hipGetLastError());
  SMFS_HIP(hipStreamSynchronize(s));
  return SMFS_OK;
}

}  // namespace smfs
