// gfx950 kernels of the one-body preconditioned MFS matrix-vector product
// and of the GMRES / post-processing steps around it.
//
// Layout (all in HBM): targets T x 3 and sources S x 3 (positions,
// strengths) as 24-byte records; sources packed by kind (Stokeslets,
// rotlets, potential dipoles), sphere-major inside a kind.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace smfs {

namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kTileSrc = 256;  // sources staged in LDS per pass

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*sh)[kWavesPerBlock]) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = wave_sum(v[q]);
    if (lane == 0) sh[q][wave] = s;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) s += sh[threadIdx.x][w];
    sh[threadIdx.x][0] = s;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = sh[q][0];
}

// 1/sqrt(x) in FP64: the hardware estimate (about 24 correct bits) refined
// by one Newton step y <- y + (y/2)(1 - x y^2), which leaves a relative
// error of 1.5 e^2 (about 4e-15).
__device__ __forceinline__ double rsqrt_f64(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double h = fma(-x * y, y, 1.0);
  return fma(0.5 * y, h, y);
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ---------------------------------------------------------------------------
// Direct sum, FP64.  One wave owns a tile of up to kTpl*64 targets of one
// sphere (or of free points when the tile's sphere is -1); the four waves
// of a block share each LDS-staged pass of 256 sources.  blockIdx.y picks a
// contiguous slice of the packed source range (split over sources).

// Stokeslet: u += (f + r (r.f)/|r|^2) / |r|, written as ri (f + r t) with
// t = (r.f) ri^2 so that a pair costs 21 VALU operations plus one rsq.
template <int kTpl>
__device__ __forceinline__ void pair_s(const double2 &q0, const double2 &q1, const double2 &q2,
                                       double tx, double ty, double tz, double &ax, double &ay,
                                       double &az) {
  const double rx = tx - q0.x, ry = ty - q0.y, rz = tz - q1.x;
  const double r2 = fma(rx, rx, fma(ry, ry, rz * rz));
  const double ri = rsqrt_f64(r2);
  const double rf = fma(rx, q1.y, fma(ry, q2.x, rz * q2.y));
  const double t = rf * (ri * ri);
  ax = fma(fma(rx, t, q1.y), ri, ax);
  ay = fma(fma(ry, t, q2.x), ri, ay);
  az = fma(fma(rz, t, q2.y), ri, az);
}

template <int kTpl>
__device__ __forceinline__ void body_s(const double2 (*sh)[kTileSrc], int a, int b,
                                       const double (&tx)[kTpl], const double (&ty)[kTpl],
                                       const double (&tz)[kTpl], double (&ax)[kTpl],
                                       double (&ay)[kTpl], double (&az)[kTpl]) {
  int j = a;
  for (; j + 1 < b; j += 2) {  // two sources per step: both LDS reads issued first
    const double2 a0 = sh[0][j], a1 = sh[1][j], a2 = sh[2][j];
    const double2 b0 = sh[0][j + 1], b1 = sh[1][j + 1], b2 = sh[2][j + 1];
#pragma unroll
    for (int p = 0; p < kTpl; ++p) {
      pair_s<kTpl>(a0, a1, a2, tx[p], ty[p], tz[p], ax[p], ay[p], az[p]);
      pair_s<kTpl>(b0, b1, b2, tx[p], ty[p], tz[p], ax[p], ay[p], az[p]);
    }
  }
  if (j < b) {
    const double2 a0 = sh[0][j], a1 = sh[1][j], a2 = sh[2][j];
#pragma unroll
    for (int p = 0; p < kTpl; ++p) pair_s<kTpl>(a0, a1, a2, tx[p], ty[p], tz[p], ax[p], ay[p], az[p]);
  }
}

template <int kTpl>
__device__ __forceinline__ void body_r(const double2 (*sh)[kTileSrc], int a, int b,
                                       const double (&tx)[kTpl], const double (&ty)[kTpl],
                                       const double (&tz)[kTpl], double (&ax)[kTpl],
                                       double (&ay)[kTpl], double (&az)[kTpl]) {
  for (int j = a; j < b; ++j) {
    const double2 q0 = sh[0][j], q1 = sh[1][j], q2 = sh[2][j];
    const double t0 = q1.y, t1 = q2.x, t2 = q2.y;
#pragma unroll
    for (int p = 0; p < kTpl; ++p) {
      const double rx = tx[p] - q0.x, ry = ty[p] - q0.y, rz = tz[p] - q1.x;
      const double r2 = fma(rx, rx, fma(ry, ry, rz * rz));
      const double ri = rsqrt_f64(r2);
      const double c = ri * ri * ri;
      ax[p] = fma(c, fma(t1, rz, -t2 * ry), ax[p]);
      ay[p] = fma(c, fma(t2, rx, -t0 * rz), ay[p]);
      az[p] = fma(c, fma(t0, ry, -t1 * rx), az[p]);
    }
  }
}

template <int kTpl>
__device__ __forceinline__ void body_d(const double2 (*sh)[kTileSrc], int a, int b,
                                       const double (&tx)[kTpl], const double (&ty)[kTpl],
                                       const double (&tz)[kTpl], double (&ax)[kTpl],
                                       double (&ay)[kTpl], double (&az)[kTpl]) {
  for (int j = a; j < b; ++j) {
    const double2 q0 = sh[0][j], q1 = sh[1][j], q2 = sh[2][j];
#pragma unroll
    for (int p = 0; p < kTpl; ++p) {
      const double rx = tx[p] - q0.x, ry = ty[p] - q0.y, rz = tz[p] - q1.x;
      const double r2 = fma(rx, rx, fma(ry, ry, rz * rz));
      const double ri = rsqrt_f64(r2);
      const double ri2 = ri * ri;
      const double ri3 = ri2 * ri;
      const double rd = fma(rx, q1.y, fma(ry, q2.x, rz * q2.y));
      const double bb = 3.0 * rd * ri3 * ri2;
      ax[p] = fma(-q1.y, ri3, fma(rx, bb, ax[p]));
      ay[p] = fma(-q2.x, ri3, fma(ry, bb, ay[p]));
      az[p] = fma(-q2.y, ri3, fma(rz, bb, az[p]));
    }
  }
}

template <int kTpl, bool kFree>
__global__ __launch_bounds__(kBlock) void k_direct_f64(DirectArgs A) {
  __shared__ double2 sh[3][kTileSrc];
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t tile = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x / kWave);
  int k = -1, t0 = 0, tc = 0;
  if (tile < A.n_tiles) {
    if (!kFree) {
      const int4 tl = A.tiles[tile];
      k = tl.x;
      t0 = tl.y;
      tc = tl.z;
    } else {  // consecutive free points, no source skipped
      t0 = (int)(tile * kWave * kTpl);
      tc = (int)min<int64_t>(kWave * kTpl, A.T - t0);
    }
  }
  k = uniform(k);
  t0 = uniform(t0);
  tc = uniform(tc);

  double tx[kTpl], ty[kTpl], tz[kTpl], ax[kTpl], ay[kTpl], az[kTpl];
#pragma unroll
  for (int p = 0; p < kTpl; ++p) {
    const int i = lane + kWave * p;
    const int64_t ti = (int64_t)t0 + (i < tc ? i : 0);
    tx[p] = A.tgt[3 * ti];
    ty[p] = A.tgt[3 * ti + 1];
    tz[p] = A.tgt[3 * ti + 2];
    ax[p] = ay[p] = az[p] = 0.0;
  }

  const int64_t S = A.kb[3];
  const int64_t lo = S * blockIdx.y / A.n_splits;
  const int64_t hi = S * (blockIdx.y + 1) / A.n_splits;

  for (int kd = 0; kd < 3; ++kd) {
    const int64_t a0 = max(lo, A.kb[kd]), a1 = min(hi, A.kb[kd + 1]);
    int64_t slo = 0, shi = 0;
    if (k >= 0) {
      slo = A.meta[k].k0[kd];
      shi = slo + A.meta[k].kn[kd];
    }
    for (int64_t j0 = a0; j0 < a1; j0 += kTileSrc) {
      const int cnt = (int)min((int64_t)kTileSrc, a1 - j0);
      __syncthreads();
      if ((int)threadIdx.x < cnt) {
        const int64_t j = j0 + threadIdx.x;
        double f0 = A.str[3 * j], f1 = A.str[3 * j + 1], f2 = A.str[3 * j + 2];
        if (kd == 2) {
          f0 *= A.dscale;
          f1 *= A.dscale;
          f2 *= A.dscale;
        }
        sh[0][threadIdx.x] = make_double2(A.src[3 * j], A.src[3 * j + 1]);
        sh[1][threadIdx.x] = make_double2(A.src[3 * j + 2], f0);
        sh[2][threadIdx.x] = make_double2(f1, f2);
      }
      __syncthreads();
      if (tc == 0) continue;
      int b1 = cnt, a2 = cnt;
      if (shi > slo) {
        b1 = (int)min<int64_t>(max<int64_t>(slo - j0, 0), cnt);
        a2 = (int)min<int64_t>(max<int64_t>(shi - j0, 0), cnt);
      }
      if (kd == 0) {
        body_s<kTpl>(sh, 0, b1, tx, ty, tz, ax, ay, az);
        body_s<kTpl>(sh, a2, cnt, tx, ty, tz, ax, ay, az);
      } else if (kd == 1) {
        body_r<kTpl>(sh, 0, b1, tx, ty, tz, ax, ay, az);
        body_r<kTpl>(sh, a2, cnt, tx, ty, tz, ax, ay, az);
      } else {
        body_d<kTpl>(sh, 0, b1, tx, ty, tz, ax, ay, az);
        body_d<kTpl>(sh, a2, cnt, tx, ty, tz, ax, ay, az);
      }
    }
  }

  double *out = A.part + (int64_t)blockIdx.y * A.T * 3;
#pragma unroll
  for (int p = 0; p < kTpl; ++p) {
    const int i = lane + kWave * p;
    if (i < tc) {
      const int64_t o = 3 * ((int64_t)t0 + i);
      out[o] = ax[p];
      out[o + 1] = ay[p];
      out[o + 2] = az[p];
    }
  }
}

__global__ void k_reduce_epilogue(int64_t n3, int32_t ns, const double *__restrict__ part,
                                  const double *__restrict__ base, const double *__restrict__ sw,
                                  double c0, double *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  double acc = 0.0;
  for (int s = 0; s < ns; ++s) acc += part[(int64_t)s * n3 + i];
  double v = c0 * acc;
  if (sw) v *= sw[i / 3];
  if (base) v += base[i];
  y[i] = v;
}

// ---------------------------------------------------------------------------
// Pseudo-inverse apply: one wave per output row, a dot product of a
// contiguous factor row with a short vector.

__global__ __launch_bounds__(kBlock) void k_pinv_u(const RowTask *__restrict__ tasks, int64_t n,
                                                   const SphereMeta *__restrict__ meta,
                                                   const FactorSlot *__restrict__ fs,
                                                   const double *__restrict__ fac,
                                                   const double *__restrict__ mu,
                                                   double *__restrict__ sbuf) {
  const int64_t t = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  if (t >= n) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int k = uniform(tasks[t].sphere), j = uniform(tasks[t].row);
  const SphereMeta &m = meta[k];
  const FactorSlot &f = fs[m.fid];
  const int rows = f.rows;
  const double *col = fac + f.u_off + (int64_t)j * rows;
  const double *x = mu + 3 * m.t0;
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  int i = lane;
  for (; i + 3 * kWave < rows; i += 4 * kWave) {
    a0 = fma(col[i], x[i], a0);
    a1 = fma(col[i + kWave], x[i + kWave], a1);
    a2 = fma(col[i + 2 * kWave], x[i + 2 * kWave], a2);
    a3 = fma(col[i + 3 * kWave], x[i + 3 * kWave], a3);
  }
  for (; i < rows; i += kWave) a0 = fma(col[i], x[i], a0);
  const double s = wave_sum((a0 + a1) + (a2 + a3));
  if (lane == 0) sbuf[m.s0 + j] = s / fac[f.sig_off + j];
}

__global__ __launch_bounds__(kBlock) void k_pinv_v(const RowTask *__restrict__ tasks, int64_t n,
                                                   const SphereMeta *__restrict__ meta,
                                                   const FactorSlot *__restrict__ fs,
                                                   const double *__restrict__ fac,
                                                   const double *__restrict__ sbuf,
                                                   double *__restrict__ lam) {
  const int64_t t = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  if (t >= n) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int k = uniform(tasks[t].sphere), r = uniform(tasks[t].row);
  const SphereMeta &m = meta[k];
  const FactorSlot &f = fs[m.fid];
  const int rank = m.rank;
  const double *row = fac + f.vt_off + (int64_t)r * f.cols;
  const double *x = sbuf + m.s0;
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  int i = lane;
  for (; i + 3 * kWave < rank; i += 4 * kWave) {
    a0 = fma(row[i], x[i], a0);
    a1 = fma(row[i + kWave], x[i + kWave], a1);
    a2 = fma(row[i + 2 * kWave], x[i + 2 * kWave], a2);
    a3 = fma(row[i + 3 * kWave], x[i + 3 * kWave], a3);
  }
  for (; i < rank; i += kWave) a0 = fma(row[i], x[i], a0);
  const double s = wave_sum((a0 + a1) + (a2 + a3));
  if (lane == 0) {
    const int jl = r / 3, c = r - 3 * (r / 3);
    int64_t p;
    if (jl < m.kn[0]) p = m.k0[0] + jl;
    else if (jl < m.kn[0] + m.kn[1]) p = m.k0[1] + (jl - m.kn[0]);
    else p = m.k0[2] + (jl - m.kn[0] - m.kn[1]);
    lam[3 * p + c] = s;
  }
}

// ---------------------------------------------------------------------------
// Right-hand side, forces/torques, residual statistics.

__global__ void k_rhs(int64_t T, const double *__restrict__ tgt, const int32_t *__restrict__ tsph,
                      const double *__restrict__ sw, const SphereMeta *__restrict__ meta,
                      const double *__restrict__ rbm, double *__restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T) return;
  const int k = tsph[i];
  const double *c = meta[k].c;
  const double *v = rbm + 6 * (int64_t)k;
  const double rx = tgt[3 * i] - c[0], ry = tgt[3 * i + 1] - c[1], rz = tgt[3 * i + 2] - c[2];
  const double s = sw[i];
  b[3 * i] = s * (v[0] + v[4] * rz - v[5] * ry);
  b[3 * i + 1] = s * (v[1] + v[5] * rx - v[3] * rz);
  b[3 * i + 2] = s * (v[2] + v[3] * ry - v[4] * rx);
}

__global__ __launch_bounds__(kBlock) void k_force_torque(const SphereMeta *__restrict__ meta,
                                                         const double *__restrict__ src,
                                                         const double *__restrict__ lam,
                                                         double *__restrict__ ft) {
  __shared__ double sh[6][kWavesPerBlock];
  const int k = blockIdx.x;
  const SphereMeta &m = meta[k];
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int j = threadIdx.x; j < m.kn[0]; j += kBlock) {
    const int64_t p = m.k0[0] + j;
    const double f0 = lam[3 * p], f1 = lam[3 * p + 1], f2 = lam[3 * p + 2];
    const double y0 = src[3 * p] - m.c[0], y1 = src[3 * p + 1] - m.c[1], y2 = src[3 * p + 2] - m.c[2];
    v[0] += f0;
    v[1] += f1;
    v[2] += f2;
    v[3] += y1 * f2 - y2 * f1;
    v[4] += y2 * f0 - y0 * f2;
    v[5] += y0 * f1 - y1 * f0;
  }
  for (int j = threadIdx.x; j < m.kn[1]; j += kBlock) {
    const int64_t p = m.k0[1] + j;
    v[3] += lam[3 * p];
    v[4] += lam[3 * p + 1];
    v[5] += lam[3 * p + 2];
  }
  block_sum<6>(v, sh);
  if (threadIdx.x < 6) ft[6 * k + threadIdx.x] = v[threadIdx.x];
}

__global__ __launch_bounds__(1024) void k_residual_stats(int64_t n, const double *__restrict__ pts,
                                                         const int32_t *__restrict__ sph,
                                                         const SphereMeta *__restrict__ meta,
                                                         const double *__restrict__ rbm,
                                                         const double *__restrict__ u,
                                                         double floor_rel, double *out) {
  __shared__ double sh[16];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  auto ubc = [&](int64_t i, double (&w)[3]) {
    const int k = sph[i];
    const double *c = meta[k].c;
    const double *v = rbm + 6 * (int64_t)k;
    const double rx = pts[3 * i] - c[0], ry = pts[3 * i + 1] - c[1], rz = pts[3 * i + 2] - c[2];
    w[0] = v[0] + v[4] * rz - v[5] * ry;
    w[1] = v[1] + v[5] * rx - v[3] * rz;
    w[2] = v[2] + v[3] * ry - v[4] * rx;
  };
  // pass 1: max |u_bc| and max |u - u_bc|
  double mb = 0.0, me = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    double w[3];
    ubc(i, w);
    const double e0 = u[3 * i] - w[0], e1 = u[3 * i + 1] - w[1], e2 = u[3 * i + 2] - w[2];
    mb = fmax(mb, sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]));
    me = fmax(me, sqrt(e0 * e0 + e1 * e1 + e2 * e2));
  }
  mb = wave_max(mb);
  me = wave_max(me);
  if (lane == 0) sh[wave] = mb;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) m = fmax(m, sh[w]);
    sh[0] = m;
  }
  __syncthreads();
  const double maxb = sh[0];
  __syncthreads();
  if (lane == 0) sh[wave] = me;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) m = fmax(m, sh[w]);
    out[1] = m;
    out[2] = maxb;
  }
  __syncthreads();
  // pass 2: masked relative residual
  double mr = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    double w[3];
    ubc(i, w);
    const double nb = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (nb > floor_rel * maxb) {
      const double e0 = u[3 * i] - w[0], e1 = u[3 * i + 1] - w[1], e2 = u[3 * i + 2] - w[2];
      mr = fmax(mr, sqrt(e0 * e0 + e1 * e1 + e2 * e2) / nb);
    }
  }
  mr = wave_max(mr);
  if (lane == 0) sh[wave] = mr;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) m = fmax(m, sh[w]);
    out[0] = m;
  }
}

__global__ __launch_bounds__(1024) void k_absmax(int64_t n, const double *__restrict__ x,
                                                 double *out) {
  __shared__ double sh[16];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, fabs(x[i]));
  m = wave_max(m);
  if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) r = fmax(r, sh[w]);
    out[0] = r;
  }
}

// ---------------------------------------------------------------------------
// Self block B = W G^(kk) (column-major), exact FP64 tensors.

__global__ void k_assemble(const double *__restrict__ tgt, const double *__restrict__ sw,
                           const double *__restrict__ src, const SphereMeta *__restrict__ meta,
                           int32_t k, double mu, double *__restrict__ B) {
  const SphereMeta &m = meta[k];
  const int64_t M = m.M, N = m.N;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  const int64_t i = idx % M, jl = idx / M;
  int kind;
  int64_t p;
  if (jl < m.kn[0]) { kind = 0; p = m.k0[0] + jl; }
  else if (jl < m.kn[0] + m.kn[1]) { kind = 1; p = m.k0[1] + (jl - m.kn[0]); }
  else { kind = 2; p = m.k0[2] + (jl - m.kn[0] - m.kn[1]); }
  const int64_t ti = m.t0 + i;
  const double r[3] = {tgt[3 * ti] - src[3 * p], tgt[3 * ti + 1] - src[3 * p + 1],
                       tgt[3 * ti + 2] - src[3 * p + 2]};
  const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
  const double rn = sqrt(r2);
  const double pi = 3.14159265358979323846;
  double K[3][3];
  if (kind == 0) {
    const double c = 1.0 / (8.0 * pi * mu * rn);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) K[a][b] = c * ((a == b ? 1.0 : 0.0) + r[a] * r[b] / r2);
  } else if (kind == 1) {
    const double c = 1.0 / (8.0 * pi * mu * rn * r2);
    K[0][0] = 0; K[0][1] = c * r[2]; K[0][2] = -c * r[1];
    K[1][0] = -c * r[2]; K[1][1] = 0; K[1][2] = c * r[0];
    K[2][0] = c * r[1]; K[2][1] = -c * r[0]; K[2][2] = 0;
  } else {
    const double r3 = rn * r2, r5 = r3 * r2;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        K[a][b] = (-(a == b ? 1.0 : 0.0) / r3 + 3.0 * r[a] * r[b] / r5) / (4.0 * pi);
  }
  const double s = sw[ti];
  const int64_t rows = 3 * M;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) B[(3 * i + a) + (3 * jl + b) * rows] = s * K[a][b];
}

// ---------------------------------------------------------------------------
// GMRES helpers.  Reductions are two-stage with a fixed order, so results
// are bitwise reproducible from run to run.

constexpr int kDotVecs = 8;

__global__ __launch_bounds__(kBlock) void k_mdot(const double *__restrict__ V, int64_t ld,
                                                 int32_t nv, const double *__restrict__ w,
                                                 int64_t n, int64_t chunk,
                                                 double *__restrict__ part, int32_t nchunks) {
  __shared__ double sh[kDotVecs][kWavesPerBlock];
  const int c = blockIdx.x;
  const int j0 = blockIdx.y * kDotVecs;
  const int64_t b = (int64_t)c * chunk, e = min(n, b + chunk);
  double acc[kDotVecs];
#pragma unroll
  for (int q = 0; q < kDotVecs; ++q) acc[q] = 0.0;
  for (int64_t i = b + threadIdx.x; i < e; i += kBlock) {
    const double wi = w[i];
#pragma unroll
    for (int q = 0; q < kDotVecs; ++q)
      if (j0 + q < nv) acc[q] = fma(V[(int64_t)(j0 + q) * ld + i], wi, acc[q]);
  }
  block_sum<kDotVecs>(acc, sh);
  if (threadIdx.x < kDotVecs && j0 + (int)threadIdx.x < nv)
    part[(int64_t)(j0 + threadIdx.x) * nchunks + c] = acc[threadIdx.x];
}

__global__ void k_mdot_final(int32_t nv, const double *__restrict__ part, int32_t nchunks,
                             double *__restrict__ h, int acc) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nv) return;
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += part[(int64_t)j * nchunks + c];
  h[j] = acc ? h[j] + s : s;
}

__global__ void k_mupdate(const double *__restrict__ V, int64_t ld, int32_t nv,
                          const double *__restrict__ h, double *__restrict__ w, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < nv; ++j) s = fma(V[(int64_t)j * ld + i], h[j], s);
  w[i] -= s;
}

__global__ void k_combine(const double *__restrict__ V, int64_t ld, int32_t nv,
                          const double *__restrict__ cf, double *__restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < nv; ++j) s = fma(V[(int64_t)j * ld + i], cf[j], s);
  x[i] += s;
}

__global__ __launch_bounds__(kBlock) void k_sumsq(const double *__restrict__ w, int64_t n,
                                                  int64_t chunk, double *__restrict__ part) {
  __shared__ double sh[1][kWavesPerBlock];
  const int64_t b = (int64_t)blockIdx.x * chunk, e = min(n, b + chunk);
  double acc[1] = {0.0};
  for (int64_t i = b + threadIdx.x; i < e; i += kBlock) acc[0] = fma(w[i], w[i], acc[0]);
  block_sum<1>(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

__global__ void k_sqrt_final(const double *__restrict__ part, int32_t nchunks, double *beta,
                             double *out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += part[c];
  s = sqrt(s);
  if (beta) beta[0] = s;
  if (out) out[0] = s;
}

__global__ void k_scale(double *__restrict__ w, int64_t n, const double *__restrict__ beta) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double b = beta[0];
  w[i] = b > 0.0 ? w[i] / b : 0.0;
}

__global__ void k_axpby(int64_t n, double a, const double *__restrict__ x, double b,
                        double *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}

__global__ void k_fill(int64_t n, double v, double *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = v;
}

__global__ void k_sub(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                      double *__restrict__ o) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = x[i] - y[i];
}

inline unsigned blocks_for(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

int64_t chunk_len(int64_t n, int32_t nchunks) { return (n + nchunks - 1) / nchunks; }

}  // namespace

int32_t mdot_chunks(int64_t n) {
  int64_t c = (n + 4095) / 4096;
  if (c < 1) c = 1;
  if (c > 512) c = 512;
  return (int32_t)c;
}

hipError_t launch_direct_f64(const DirectArgs &a, hipStream_t s) {
  if (a.n_tiles == 0) return hipSuccess;
  dim3 grid((unsigned)((a.n_tiles + kWavesPerBlock - 1) / kWavesPerBlock), (unsigned)a.n_splits);
  // free points (no tile table) get their own instantiation so that kernel
  // statistics of the product with G_hat are not mixed with flow evaluation
  if (a.tiles)
    hipLaunchKernelGGL((k_direct_f64<2, false>), grid, dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((k_direct_f64<2, true>), grid, dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_reduce_epilogue(int64_t n3, int32_t ns, const double *part, const double *base,
                                  const double *sw, double c0, double *y, hipStream_t s) {
  if (n3 == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_epilogue, dim3(blocks_for(n3)), dim3(kBlock), 0, s, n3, ns, part,
                     base, sw, c0, y);
  return hipGetLastError();
}

hipError_t launch_pinv_u(const RowTask *tasks, int64_t n, const SphereMeta *meta,
                         const FactorSlot *fs, const double *fac, const double *mu, double *sbuf,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pinv_u, dim3(blocks_for(n, kWavesPerBlock)), dim3(kBlock), 0, s, tasks, n,
                     meta, fs, fac, mu, sbuf);
  return hipGetLastError();
}

hipError_t launch_pinv_v(const RowTask *tasks, int64_t n, const SphereMeta *meta,
                         const FactorSlot *fs, const double *fac, const double *sbuf, double *lam,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pinv_v, dim3(blocks_for(n, kWavesPerBlock)), dim3(kBlock), 0, s, tasks, n,
                     meta, fs, fac, sbuf, lam);
  return hipGetLastError();
}

hipError_t launch_rhs(int64_t T, const double *tgt, const int32_t *tsph, const double *sw,
                      const SphereMeta *meta, const double *rbm, double *b, hipStream_t s) {
  if (T == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rhs, dim3(blocks_for(T)), dim3(kBlock), 0, s, T, tgt, tsph, sw, meta, rbm, b);
  return hipGetLastError();
}

hipError_t launch_force_torque(int32_t P, const SphereMeta *meta, const double *src,
                               const double *lam, double *ft, hipStream_t s) {
  if (P == 0) return hipSuccess;
  hipLaunchKernelGGL(k_force_torque, dim3(P), dim3(kBlock), 0, s, meta, src, lam, ft);
  return hipGetLastError();
}

hipError_t launch_residual_stats(int64_t n, const double *pts, const int32_t *sph,
                                 const SphereMeta *meta, const double *rbm, const double *u,
                                 double floor_rel, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_residual_stats, dim3(1), dim3(1024), 0, s, n, pts, sph, meta, rbm, u,
                     floor_rel, out);
  return hipGetLastError();
}

hipError_t launch_absmax(int64_t n, const double *x, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_absmax, dim3(1), dim3(1024), 0, s, n, x, out);
  return hipGetLastError();
}

hipError_t launch_assemble_block(const double *tgt, const double *sw, const double *src,
                                 const SphereMeta *meta, int32_t k, int64_t M, int64_t N, double mu,
                                 double *B, hipStream_t s) {
  const int64_t n = M * N;
  hipLaunchKernelGGL(k_assemble, dim3(blocks_for(n)), dim3(kBlock), 0, s, tgt, sw, src, meta, k,
                     mu, B);
  return hipGetLastError();
}

hipError_t launch_mdot(const double *V, int64_t ld, int32_t nv, const double *w, int64_t n,
                       double *part, int32_t nchunks, double *h, bool acc, hipStream_t s) {
  if (nv <= 0) return hipSuccess;
  const int64_t chunk = chunk_len(n, nchunks);
  dim3 grid((unsigned)nchunks, (unsigned)((nv + kDotVecs - 1) / kDotVecs));
  hipLaunchKernelGGL(k_mdot, grid, dim3(kBlock), 0, s, V, ld, nv, w, n, chunk, part, nchunks);
  hipLaunchKernelGGL(k_mdot_final, dim3(blocks_for(nv)), dim3(kBlock), 0, s, nv, part, nchunks, h,
                     acc ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_mupdate(const double *V, int64_t ld, int32_t nv, const double *h, double *w,
                          int64_t n, hipStream_t s) {
  if (nv <= 0 || n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mupdate, dim3(blocks_for(n)), dim3(kBlock), 0, s, V, ld, nv, h, w, n);
  return hipGetLastError();
}

hipError_t launch_combine(const double *V, int64_t ld, int32_t nv, const double *c, double *x,
                          int64_t n, hipStream_t s) {
  if (nv <= 0 || n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_combine, dim3(blocks_for(n)), dim3(kBlock), 0, s, V, ld, nv, c, x, n);
  return hipGetLastError();
}

hipError_t launch_norm2(const double *w, int64_t n, double *part, int32_t nchunks, double *out,
                        hipStream_t s) {
  const int64_t chunk = chunk_len(n, nchunks);
  hipLaunchKernelGGL(k_sumsq, dim3(nchunks), dim3(kBlock), 0, s, w, n, chunk, part);
  hipLaunchKernelGGL(k_sqrt_final, dim3(1), dim3(64), 0, s, part, nchunks, (double *)nullptr, out);
  return hipGetLastError();
}

hipError_t launch_norm_scale(double *w, int64_t n, double *part, int32_t nchunks, double *beta,
                             double *out, hipStream_t s) {
  const int64_t chunk = chunk_len(n, nchunks);
  hipLaunchKernelGGL(k_sumsq, dim3(nchunks), dim3(kBlock), 0, s, w, n, chunk, part);
  hipLaunchKernelGGL(k_sqrt_final, dim3(1), dim3(64), 0, s, part, nchunks, beta, out);
  hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, s, w, n, beta);
  return hipGetLastError();
}

hipError_t launch_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpby, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, a, x, b, y);
  return hipGetLastError();
}

hipError_t launch_fill(int64_t n, double v, double *y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, v, y);
  return hipGetLastError();
}

hipError_t launch_sub(int64_t n, const double *x, const double *y, double *out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sub, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, x, y, out);
  return hipGetLastError();
}

}  // namespace smfs
