// gfx950 kernels of the one-body preconditioned MFS matrix-vector product
// and of the GMRES / post-processing steps around it.
//
// Layout (all in HBM): targets T x 3 and sources S x 3 (positions,
// strengths) as 24-byte records; sources packed by kind (Stokeslets,
// rotlets, potential dipoles), sphere-major inside a kind.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace smfs {

namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
// occupancy target of the FP64 direct sum (waves per SIMD; sets its VGPR
// budget: 5 fits the pair loop in 90 VGPRs without spills and measured
// faster than 4 or 6)
#ifndef SMFS_DIRECT_WAVES
#define SMFS_DIRECT_WAVES 5
#endif

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

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ---------------------------------------------------------------------------
// Direct sum, FP64.  One wave owns a tile of up to 64*kTpl targets of one
// sphere (or of free points).  Sources are streamed with wave-uniform
// addresses, so they arrive through scalar loads into SGPRs and every VALU
// instruction of a pair reads at most one of them: no LDS staging and no
// barriers.  The sources visited are a list of ranges of the packed source
// array (per precision mode); blockIdx.y takes a contiguous slice of the
// concatenated ranges (split over sources), and the tile's own sphere is
// cut out of each range (the identity self blocks of G_hat).

// 2/sqrt(x) in FP64: the hardware estimate y of 1/sqrt(x) (about 24 correct
// bits) refined by one Newton step y (3 - x y^2) / 2 without its halving
// (3 VALU operations besides the rsq instead of 4); relative error
// 1.5 e^2 + a few ulp, about 4e-15.
__device__ __forceinline__ double rsq2_f64(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return y * fma(-x, y * y, 3.0);
}

// f/4 for a wave-uniform f, as integer operations on the high word (they
// stay on the scalar unit): the exponent field E becomes E - min(E, 2).
// Exact for normal results; zero stays zero, and |f| below 2^-1020 gives a
// value off by less than 2^-1022.
__device__ __forceinline__ double quarter(double f) {
  typedef unsigned Words __attribute__((ext_vector_type(2)));  // (low, high)
  Words w = __builtin_bit_cast(Words, f);
  w.y -= min(w.y & 0x7ff00000u, 0x00200000u);
  return __builtin_bit_cast(double, w);
}

// The pair functions below add TWICE the velocity of one source (the factor
// of two is what rsq2_f64 leaves; the tile's sums are halved once at the
// end).
//
// Stokeslet: u = (f + r (r.f)/|r|^2) / |r|.  With Y = 2/|r| and g = f/4:
// 2u = Y (f + r t), t = (r.g) Y^2 = (r.f)/|r|^2 -- 20 VALU operations plus
// one rsq per pair.
__device__ __forceinline__ void pair_s(double sx, double sy, double sz, double fx, double fy,
                                       double fz, double gx, double gy, double gz, double tx,
                                       double ty, double tz, double &ax, double &ay, double &az) {
  const double rx = tx - sx, ry = ty - sy, rz = tz - sz;
  const double r2 = fma(rx, rx, fma(ry, ry, rz * rz));
  const double Y = rsq2_f64(r2);
  const double rg = fma(rx, gx, fma(ry, gy, rz * gz));
  const double t = rg * (Y * Y);
  ax = fma(fma(rx, t, fx), Y, ax);
  ay = fma(fma(ry, t, fy), Y, ay);
  az = fma(fma(rz, t, fz), Y, az);
}

// Rotlet: u = (t x r) / |r|^3; 2/|r|^3 = Y^3/4.
__device__ __forceinline__ void pair_r(double sx, double sy, double sz, double t0, double t1,
                                       double t2, double tx, double ty, double tz, double &ax,
                                       double &ay, double &az) {
  const double rx = tx - sx, ry = ty - sy, rz = tz - sz;
  const double r2 = fma(rx, rx, fma(ry, ry, rz * rz));
  const double Y = rsq2_f64(r2);
  const double c = (0.25 * Y) * (Y * Y);
  ax = fma(c, fma(t1, rz, -t2 * ry), ax);
  ay = fma(c, fma(t2, rx, -t0 * rz), ay);
  az = fma(c, fma(t0, ry, -t1 * rx), az);
}

// Potential dipole (strength pre-multiplied by 2 mu so that the common
// factor 1/(8 pi mu) applies): u = -d/|r|^3 + 3 r (r.d)/|r|^5;
// 2/|r|^3 = Y^3/4 and 6/|r|^5 = (3/4) (Y^3/4) Y^2.
__device__ __forceinline__ void pair_d(double sx, double sy, double sz, double d0, double d1,
                                       double d2, double tx, double ty, double tz, double &ax,
                                       double &ay, double &az) {
  const double rx = tx - sx, ry = ty - sy, rz = tz - sz;
  const double r2 = fma(rx, rx, fma(ry, ry, rz * rz));
  const double Y = rsq2_f64(r2);
  const double Y2 = Y * Y;
  const double c3 = 0.25 * (Y2 * Y);
  const double rd = fma(rx, d0, fma(ry, d1, rz * d2));
  const double bb = (0.75 * rd) * c3 * Y2;
  ax = fma(-d0, c3, fma(rx, bb, ax));
  ay = fma(-d1, c3, fma(ry, bb, ay));
  az = fma(-d2, c3, fma(rz, bb, az));
}

template <int kTpl>
struct Acc {
  double tx[kTpl], ty[kTpl], tz[kTpl], ax[kTpl], ay[kTpl], az[kTpl];
};

// Sources [j0, j1) of one kind; j0, j1 wave-uniform.
// Source positions and strengths do not change during a direct-sum launch;
// reading them through the constant address space lets the compiler use
// scalar loads for the wave-uniform addresses also where the pointers come
// from a descriptor in memory (the serving kernel), not from kernel arguments.
typedef __attribute__((address_space(4))) const double *ConstPtr;

template <int kTpl, int kKind, bool kScaleD>
__device__ __forceinline__ void run_sources(const double *__restrict__ src_,
                                            const double *__restrict__ str_, double dscale,
                                            int64_t j0_, int64_t j1_, Acc<kTpl> &A) {
  const ConstPtr src = (ConstPtr)src_, str = (ConstPtr)str_;
  // source indices fit in 32 bits; wave-uniform bounds keep the loop test on
  // the scalar unit
  int j = uniform((int)j0_);
  const int j1 = uniform((int)j1_);
  // two Stokeslets per step (rotlet and dipole ranges are short: one per step)
  for (; kKind == 0 && j + 1 < j1; j += 2) {
    const ConstPtr p0 = src + 3 * j, q0 = str + 3 * j;
    const double s0x = p0[0], s0y = p0[1], s0z = p0[2], s1x = p0[3], s1y = p0[4], s1z = p0[5];
    double f0x = q0[0], f0y = q0[1], f0z = q0[2], f1x = q0[3], f1y = q0[4], f1z = q0[5];
    if (kKind == 2 && kScaleD) {
      f0x *= dscale; f0y *= dscale; f0z *= dscale;
      f1x *= dscale; f1y *= dscale; f1z *= dscale;
    }
    const double g0x = quarter(f0x), g0y = quarter(f0y), g0z = quarter(f0z);
    const double g1x = quarter(f1x), g1y = quarter(f1y), g1z = quarter(f1z);
#pragma unroll
    for (int p = 0; p < kTpl; ++p) {
      if (kKind == 0) {
        pair_s(s0x, s0y, s0z, f0x, f0y, f0z, g0x, g0y, g0z, A.tx[p], A.ty[p], A.tz[p], A.ax[p],
               A.ay[p], A.az[p]);
        pair_s(s1x, s1y, s1z, f1x, f1y, f1z, g1x, g1y, g1z, A.tx[p], A.ty[p], A.tz[p], A.ax[p],
               A.ay[p], A.az[p]);
      } else if (kKind == 1) {
        pair_r(s0x, s0y, s0z, f0x, f0y, f0z, A.tx[p], A.ty[p], A.tz[p], A.ax[p], A.ay[p], A.az[p]);
        pair_r(s1x, s1y, s1z, f1x, f1y, f1z, A.tx[p], A.ty[p], A.tz[p], A.ax[p], A.ay[p], A.az[p]);
      } else {
        pair_d(s0x, s0y, s0z, f0x, f0y, f0z, A.tx[p], A.ty[p], A.tz[p], A.ax[p], A.ay[p], A.az[p]);
        pair_d(s1x, s1y, s1z, f1x, f1y, f1z, A.tx[p], A.ty[p], A.tz[p], A.ax[p], A.ay[p], A.az[p]);
      }
    }
  }
  for (; j < j1; ++j) {
    const ConstPtr p0 = src + 3 * j, q0 = str + 3 * j;
    const double sx = p0[0], sy = p0[1], sz = p0[2];
    double fx = q0[0], fy = q0[1], fz = q0[2];
    if (kKind == 2 && kScaleD) { fx *= dscale; fy *= dscale; fz *= dscale; }
    const double gx = quarter(fx), gy = quarter(fy), gz = quarter(fz);
#pragma unroll
    for (int p = 0; p < kTpl; ++p) {
      if (kKind == 0)
        pair_s(sx, sy, sz, fx, fy, fz, gx, gy, gz, A.tx[p], A.ty[p], A.tz[p], A.ax[p], A.ay[p],
               A.az[p]);
      else if (kKind == 1) pair_r(sx, sy, sz, fx, fy, fz, A.tx[p], A.ty[p], A.tz[p], A.ax[p], A.ay[p], A.az[p]);
      else pair_d(sx, sy, sz, fx, fy, fz, A.tx[p], A.ty[p], A.tz[p], A.ax[p], A.ay[p], A.az[p]);
    }
  }
}

// Dipole strengths of a product with G_hat arrive pre-multiplied by 2 mu
// (written so by the pseudo-inverse apply); free-point evaluation takes
// physical strengths and scales them here.
template <int kTpl, bool kScaleD>
__device__ __forceinline__ void run_block(int block, const DirectArgs &A, int64_t j0, int64_t j1,
                                          Acc<kTpl> &acc) {
  if (j0 >= j1) return;
  if (block <= 1) run_sources<kTpl, 0, kScaleD>(A.src, A.str, A.dscale, j0, j1, acc);
  else if (block == 2) run_sources<kTpl, 1, kScaleD>(A.src, A.str, A.dscale, j0, j1, acc);
  else run_sources<kTpl, 2, kScaleD>(A.src, A.str, A.dscale, j0, j1, acc);
}

// Sources [j0, j1) of one kind for the target slots with on[p] set only:
// in a tile that spans several spheres, each member sphere's own sources
// reach the targets of the other members.  One source per step; a masked
// slot's new sum is discarded by a select, so it stays unchanged bitwise.
template <int kTpl, int kKind, bool kScaleD>
__device__ __forceinline__ void run_sources_masked(const double *__restrict__ src_,
                                                   const double *__restrict__ str_, double dscale,
                                                   int64_t j0_, int64_t j1_, Acc<kTpl> &A,
                                                   const bool (&on)[kTpl]) {
  const ConstPtr src = (ConstPtr)src_, str = (ConstPtr)str_;
  const int j1 = uniform((int)j1_);
  for (int j = uniform((int)j0_); j < j1; ++j) {
    const ConstPtr p0 = src + 3 * j, q0 = str + 3 * j;
    const double sx = p0[0], sy = p0[1], sz = p0[2];
    double fx = q0[0], fy = q0[1], fz = q0[2];
    if (kKind == 2 && kScaleD) { fx *= dscale; fy *= dscale; fz *= dscale; }
    const double gx = quarter(fx), gy = quarter(fy), gz = quarter(fz);
#pragma unroll
    for (int p = 0; p < kTpl; ++p) {
      double bx = A.ax[p], by = A.ay[p], bz = A.az[p];
      if (kKind == 0) pair_s(sx, sy, sz, fx, fy, fz, gx, gy, gz, A.tx[p], A.ty[p], A.tz[p], bx, by, bz);
      else if (kKind == 1) pair_r(sx, sy, sz, fx, fy, fz, A.tx[p], A.ty[p], A.tz[p], bx, by, bz);
      else pair_d(sx, sy, sz, fx, fy, fz, A.tx[p], A.ty[p], A.tz[p], bx, by, bz);
      A.ax[p] = on[p] ? bx : A.ax[p];
      A.ay[p] = on[p] ? by : A.ay[p];
      A.az[p] = on[p] ? bz : A.az[p];
    }
  }
}

template <int kTpl, bool kScaleD>
__device__ __forceinline__ void run_block_masked(int block, const DirectArgs &A, int64_t j0, int64_t j1,
                                                 Acc<kTpl> &acc, const bool (&on)[kTpl]) {
  if (j0 >= j1) return;
  if (block <= 1) run_sources_masked<kTpl, 0, kScaleD>(A.src, A.str, A.dscale, j0, j1, acc, on);
  else if (block == 2) run_sources_masked<kTpl, 1, kScaleD>(A.src, A.str, A.dscale, j0, j1, acc, on);
  else run_sources_masked<kTpl, 2, kScaleD>(A.src, A.str, A.dscale, j0, j1, acc, on);
}

// One wave: tile `tile` of A, source split `split`.  A tile holds up to
// 64 kTpl consecutive targets, which may belong to consecutive spheres
// ka..kb (every wave then has a full tile of work, whatever the node count
// of a sphere).  The sources of ka..kb are contiguous in every block
// (sphere-major packing): the main loops cut them out, and a masked pass
// gives each member's sources to the other members' targets.
template <int kTpl, bool kFree>
__device__ __forceinline__ void direct_wave(const DirectArgs &A, int64_t tile, int64_t split) {
  const int lane = threadIdx.x & (kWave - 1);
  int ka = -1, kb = -1, t0 = 0, tc = 0;
  if (tile < A.n_tiles) {
    if (!kFree) {
      const int4 tl = A.tiles[tile];
      ka = tl.x;
      t0 = tl.y;
      tc = tl.z;
      kb = tl.w;
    } else {  // consecutive free points, no source skipped
      t0 = (int)(tile * kWave * kTpl);
      tc = (int)min<int64_t>(kWave * kTpl, A.T - t0);
    }
  }
  ka = uniform(ka);
  kb = uniform(kb);
  t0 = uniform(t0);
  tc = uniform(tc);
  if (tc <= 0) return;  // whole wave idle (no barriers in this kernel)
  int own[kTpl];        // sphere of each target slot (multi-sphere tiles)
#pragma unroll
  for (int p = 0; p < kTpl; ++p) {
    const int i = lane + kWave * p;
    own[p] = (!kFree && ka != kb && i < tc) ? A.tsph[t0 + i] : -1;
  }

  Acc<kTpl> acc;
#pragma unroll
  for (int p = 0; p < kTpl; ++p) {
    const int i = lane + kWave * p;
    const int64_t ti = (int64_t)t0 + (i < tc ? i : 0);
    acc.tx[p] = A.tgt[3 * ti];
    acc.ty[p] = A.tgt[3 * ti + 1];
    acc.tz[p] = A.tgt[3 * ti + 2];
    acc.ax[p] = acc.ay[p] = acc.az[p] = 0.0;
  }

  const int64_t L = A.range_total;
  const int64_t lo = L * split / A.n_splits;
  const int64_t hi = L * (split + 1) / A.n_splits;
  int64_t pos = 0;
  for (int r = 0; r < A.n_ranges && pos < hi; ++r) {
    const SrcRange R = A.ranges[r];
    const int64_t len = R.end - R.begin;
    const int64_t a = max<int64_t>(lo - pos, 0), b = min<int64_t>(hi - pos, len);
    pos += len;
    if (a >= b) continue;
    const int64_t j0 = R.begin + a, j1 = R.begin + b;
    if (ka >= 0) {  // cut the tile's spheres out of this block
      const int64_t s0 = A.meta[ka].k0[R.block], s1 = A.meta[kb].k0[R.block] + A.meta[kb].kn[R.block];
      run_block<kTpl, kFree>(R.block, A, j0, min(j1, s0), acc);
      run_block<kTpl, kFree>(R.block, A, max(j0, s1), j1, acc);
      for (int q = ka; q <= kb && ka != kb; ++q) {
        const int64_t m0 = A.meta[q].k0[R.block], m1 = m0 + A.meta[q].kn[R.block];
        bool on[kTpl];
#pragma unroll
        for (int p = 0; p < kTpl; ++p) on[p] = own[p] != q;
        run_block_masked<kTpl, kFree>(R.block, A, max(j0, m0), min(j1, m1), acc, on);
      }
    } else {
      run_block<kTpl, kFree>(R.block, A, j0, j1, acc);
    }
  }

  double *out = A.part + split * A.T * 3;
#pragma unroll
  for (int p = 0; p < kTpl; ++p) {
    const int i = lane + kWave * p;
    if (i < tc) {
      const int64_t o = 3 * ((int64_t)t0 + i);
      out[o] = 0.5 * acc.ax[p];  // the pair functions add twice the velocity
      out[o + 1] = 0.5 * acc.ay[p];
      out[o + 2] = 0.5 * acc.az[p];
    }
  }
}

template <int kTpl, bool kFree>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(SMFS_DIRECT_WAVES, 8))) void k_direct_f64(DirectArgs A) {
  const int64_t tile = (int64_t)blockIdx.x * kWavesPerBlock + uniform(threadIdx.x / kWave);
  direct_wave<kTpl, kFree>(A, tile, blockIdx.y);
}

// ---------------------------------------------------------------------------
// Direct sum, FP32 (mixed precision): Stokeslets of contact-free spheres
// only (every pair with such a source is well separated: its sphere has no
// neighbour closer than the image cutoff).  Coordinates are relative to
// each sphere's centre; the centre offset of every source sphere is formed
// in FP64 and rounded once, so the FP32 separation keeps its relative
// accuracy at every distance.  Accumulation in FP32.

typedef __attribute__((address_space(4))) const float *ConstPtr32;

// One far-field pair in FP32 (no refinement of the hardware rsq: about one
// ulp, enough for the FP32 sum).
template <int kTpl>
__device__ __forceinline__ void far_pair(float sx, float sy, float sz, float fx, float fy, float fz,
                                         const float (&ux)[kTpl], const float (&uy)[kTpl],
                                         const float (&uz)[kTpl], float (&ax)[kTpl],
                                         float (&ay)[kTpl], float (&az)[kTpl]) {
#pragma unroll
  for (int p = 0; p < kTpl; ++p) {
    const float rx = ux[p] - sx, ry = uy[p] - sy, rz = uz[p] - sz;
    const float r2 = fmaf(rx, rx, fmaf(ry, ry, rz * rz));
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float rf = fmaf(rx, fx, fmaf(ry, fy, rz * fz));
    const float t = rf * (ri * ri);
    ax[p] = fmaf(fmaf(rx, t, fx), ri, ax[p]);
    ay[p] = fmaf(fmaf(ry, t, fy), ri, ay[p]);
    az[p] = fmaf(fmaf(rz, t, fz), ri, az[p]);
  }
}

// One wave of the FP32 far-field sum: tile `tile` of A, split `split`.
template <int kTpl>
__device__ __forceinline__ void far_wave(const Far32Args &A, int64_t tile, int split) {
  const int lane = threadIdx.x & (kWave - 1);
  if (tile >= A.n_tiles) return;
  const int4 tl = A.tiles[tile];
  const int k = uniform(tl.x), t0 = uniform(tl.y), tc = uniform(tl.z);
  if (tc <= 0) return;
  float tx[kTpl], ty[kTpl], tz[kTpl], ax[kTpl], ay[kTpl], az[kTpl];
#pragma unroll
  for (int p = 0; p < kTpl; ++p) {
    const int i = lane + kWave * p;
    const int64_t ti = (int64_t)t0 + (i < tc ? i : 0);
    tx[p] = A.tgt32[3 * ti];
    ty[p] = A.tgt32[3 * ti + 1];
    tz[p] = A.tgt32[3 * ti + 2];
    ax[p] = ay[p] = az[p] = 0.f;
  }
  const ConstPtr32 src = (ConstPtr32)A.src32, str = (ConstPtr32)A.str32;
  const double ckx = A.centers[3 * k], cky = A.centers[3 * k + 1], ckz = A.centers[3 * k + 2];
  const int q0 = uniform((int)((int64_t)A.n_free * split / A.n_splits));
  const int q1 = uniform((int)((int64_t)A.n_free * (split + 1) / A.n_splits));
  const int np = A.n_proxy;
  for (int q = q0; q < q1; ++q) {
    const int ks = A.free_ids[q];
    if (ks == k) continue;
    const float dx = (float)(A.centers[3 * ks] - ckx), dy = (float)(A.centers[3 * ks + 1] - cky),
                dz = (float)(A.centers[3 * ks + 2] - ckz);
    float ux[kTpl], uy[kTpl], uz[kTpl];
#pragma unroll
    for (int p = 0; p < kTpl; ++p) {
      ux[p] = tx[p] - dx;
      uy[p] = ty[p] - dy;
      uz[p] = tz[p] - dz;
    }
    // proxy indices fit in 32 bits (wave-uniform: the loop test stays on
    // the scalar unit); two sources per step
    int j = uniform(ks * np);
    const int j1 = j + np;
    for (; j + 1 < j1; j += 2) {
      const ConstPtr32 ps = src + 3 * j, pf = str + 3 * j;
      const float s0x = ps[0], s0y = ps[1], s0z = ps[2], s1x = ps[3], s1y = ps[4], s1z = ps[5];
      const float f0x = pf[0], f0y = pf[1], f0z = pf[2], f1x = pf[3], f1y = pf[4], f1z = pf[5];
      far_pair<kTpl>(s0x, s0y, s0z, f0x, f0y, f0z, ux, uy, uz, ax, ay, az);
      far_pair<kTpl>(s1x, s1y, s1z, f1x, f1y, f1z, ux, uy, uz, ax, ay, az);
    }
    if (j < j1) {
      const ConstPtr32 ps = src + 3 * j, pf = str + 3 * j;
      far_pair<kTpl>(ps[0], ps[1], ps[2], pf[0], pf[1], pf[2], ux, uy, uz, ax, ay, az);
    }
  }
  float *out = A.part32 + (int64_t)split * A.T * 3;
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

template <int kTpl>
__global__ __launch_bounds__(kBlock) void k_far_f32(Far32Args A) {
  const int64_t tile = (int64_t)blockIdx.x * kWavesPerBlock + uniform(threadIdx.x / kWave);
  far_wave<kTpl>(A, tile, blockIdx.y);
}

__global__ void k_reduce_epilogue(int64_t n3, int32_t ns, const double *__restrict__ part,
                                  int32_t ns32, const float *__restrict__ part32,
                                  const double *__restrict__ base, const double *__restrict__ sw,
                                  double c0, double *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  double acc = 0.0;
  for (int s = 0; s < ns; ++s) acc += part[(int64_t)s * n3 + i];
  for (int s = 0; s < ns32; ++s) acc += (double)part32[(int64_t)s * n3 + i];
  double v = c0 * acc;
  if (sw) v *= sw[i / 3];
  if (base) v += base[i];
  y[i] = v;
}

// ---------------------------------------------------------------------------
// Equivalent-source far field (the SMFS_MIXED_EQ product).  For a target
// sphere k and a contact-free source sphere k' at centre separation of at
// least eq_separation radii, the field of the N proxy Stokeslets of k' is
// replaced by that of n_eq equivalent Stokeslets q = E lambda_hat_k' (E
// fitted in FP64 at set-up on a check sphere around k'; the same for every
// contact-free sphere).  Pairs with a contact-free source closer than that
// (the near list of k) stay exact, in FP64.  The equivalent strengths are
// of the size of the field itself, not of the proxies' cancelling
// strengths, so their FP32 sum keeps FP32's relative accuracy.

// q32[q][r] = (float) sum_i E[r + i rows] lambda_hat(proxies of free sphere q)[i]:
// one thread per row r and four spheres; the strengths are wave-uniform.
__global__ __launch_bounds__(256) void k_eq_strengths(const double *__restrict__ E, int32_t rows, int32_t cols,
                                                      const double *__restrict__ lam,
                                                      const SphereMeta *__restrict__ meta,
                                                      const int32_t *__restrict__ free_ids, int32_t n_free,
                                                      float *__restrict__ q32) {
  constexpr int kQ = 4;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int qb = blockIdx.y * kQ;
  ConstPtr l[kQ];
#pragma unroll
  for (int u = 0; u < kQ; ++u) {
    const int q = min(qb + u, n_free - 1);
    const int ks = uniform(free_ids[q]);
    l[u] = (ConstPtr)(lam + 3 * meta[ks].k0[0]);
  }
  double acc[kQ] = {0.0, 0.0, 0.0, 0.0};
  const int rr = r < rows ? r : 0;
  for (int i = 0; i < cols; ++i) {
    const double e = E[(int64_t)i * rows + rr];
#pragma unroll
    for (int u = 0; u < kQ; ++u) acc[u] = fma(e, l[u][i], acc[u]);
  }
  if (r >= rows) return;
#pragma unroll
  for (int u = 0; u < kQ; ++u)
    if (qb + u < n_free) q32[(int64_t)(qb + u) * rows + r] = (float)acc[u];
}

// A slot that a source sphere must not reach is moved to kOffSlot: its
// squared distance to every equivalent point overflows to +inf, rsq gives
// +0 and the pair adds exactly 0 (the projection r.f stays finite for any
// strength below 1e18), so every slot runs the same loop.
constexpr float kOffSlot = 1e20f;

// The n_eq equivalent sources of one sphere (points pts relative to its
// centre, strengths str) at the slots' targets ux (relative to the same
// centre); two sources per step, the next step's points and strengths
// loaded (wave-uniform, into scalar registers) while this step computes.
template <int kTpl>
__device__ __forceinline__ void eq_sphere(ConstPtr32 pts, ConstPtr32 str, int ne, const float (&ux)[kTpl],
                                          const float (&uy)[kTpl], const float (&uz)[kTpl], float (&ax)[kTpl],
                                          float (&ay)[kTpl], float (&az)[kTpl]) {
  int j = 0;
  if (ne >= 2) {
    float c[12];   // points of sources j, j + 1, then their strengths
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      c[u] = pts[u];
      c[6 + u] = str[u];
    }
    for (; j + 3 < ne; j += 2) {
      const ConstPtr32 ps = pts + 3 * (j + 2), pf = str + 3 * (j + 2);
      float nx[12];
#pragma unroll
      for (int u = 0; u < 6; ++u) {
        nx[u] = ps[u];
        nx[6 + u] = pf[u];
      }
      far_pair<kTpl>(c[0], c[1], c[2], c[6], c[7], c[8], ux, uy, uz, ax, ay, az);
      far_pair<kTpl>(c[3], c[4], c[5], c[9], c[10], c[11], ux, uy, uz, ax, ay, az);
#pragma unroll
      for (int u = 0; u < 12; ++u) c[u] = nx[u];
    }
    far_pair<kTpl>(c[0], c[1], c[2], c[6], c[7], c[8], ux, uy, uz, ax, ay, az);
    far_pair<kTpl>(c[3], c[4], c[5], c[9], c[10], c[11], ux, uy, uz, ax, ay, az);
    j += 2;
  }
  if (j < ne) {
    const ConstPtr32 ps = pts + 3 * j, pf = str + 3 * j;
    far_pair<kTpl>(ps[0], ps[1], ps[2], pf[0], pf[1], pf[2], ux, uy, uz, ax, ay, az);
  }
}

// One wave of the FP32 equivalent-source sum: tile `tile` and split
// `split` of the contact-free spheres (free-index order).  A tile holds up
// to 64 kTpl consecutive targets, which may belong to consecutive spheres,
// so that every wave has a full tile whatever a sphere's node count.  Each
// slot skips its own sphere and the near list of its sphere, walking that
// ascending list beside the sphere loop; a slot that skips a source sphere
// summed for others is moved out of its reach (kOffSlot).  A slot's
// coordinates relative to a source sphere's centre are formed in FP64 and
// rounded once.
template <int kTpl>
__device__ __forceinline__ void far_eq_wave(const EqArgs &A, int64_t tile, int split) {
  const int lane = threadIdx.x & (kWave - 1);
  if (tile >= A.n_tiles) return;
  const int4 tl = A.tiles[tile];
  const int t0 = uniform(tl.y), tc = uniform(tl.z);
  if (tc <= 0) return;
  const int q0 = uniform((int)((int64_t)A.n_free * split / A.n_splits));
  const int q1 = uniform((int)((int64_t)A.n_free * (split + 1) / A.n_splits));
  double tx[kTpl], ty[kTpl], tz[kTpl];  // targets, absolute
  float ax[kTpl], ay[kTpl], az[kTpl];
  int own[kTpl], e[kTpl], next[kTpl];
#pragma unroll
  for (int p = 0; p < kTpl; ++p) {
    const int i = lane + kWave * p;
    const int64_t ti = (int64_t)t0 + (i < tc ? i : 0);
    tx[p] = A.tgt[3 * ti];
    ty[p] = A.tgt[3 * ti + 1];
    tz[p] = A.tgt[3 * ti + 2];
    ax[p] = ay[p] = az[p] = 0.f;
    const int k = A.tsph[ti];
    own[p] = k;
    // the near list of k is ascending: skip its entries below q0
    e[p] = A.near_off[k];
    const int e1 = A.near_off[k + 1];
    while (e[p] < e1 && A.near_idx[e[p]] < q0) ++e[p];
    next[p] = e[p] < e1 ? A.near_idx[e[p]] : 0x7fffffff;
  }
  const ConstPtr32 pts = (ConstPtr32)A.eqpt32;
  const int ne = A.n_eq;
  for (int q = q0; q < q1; ++q) {
    const int ks = uniform(A.free_ids[q]);
    bool on[kTpl];
    bool any_on = false;
#pragma unroll
    for (int p = 0; p < kTpl; ++p) {
      const bool near = q == next[p];
      if (near) {
        ++e[p];
        next[p] = e[p] < A.near_off[own[p] + 1] ? A.near_idx[e[p]] : 0x7fffffff;
      }
      on[p] = !near && ks != own[p];
      any_on = any_on || on[p];
    }
    if (!__any(any_on)) continue;
    const double sx = A.centers[3 * ks], sy = A.centers[3 * ks + 1], sz = A.centers[3 * ks + 2];
    float ux[kTpl], uy[kTpl], uz[kTpl];
#pragma unroll
    for (int p = 0; p < kTpl; ++p) {
      ux[p] = on[p] ? (float)(tx[p] - sx) : kOffSlot;
      uy[p] = on[p] ? (float)(ty[p] - sy) : kOffSlot;
      uz[p] = on[p] ? (float)(tz[p] - sz) : kOffSlot;
    }
    const ConstPtr32 str = (ConstPtr32)(A.q32 + (int64_t)q * 3 * ne);
    eq_sphere<kTpl>(pts, str, ne, ux, uy, uz, ax, ay, az);
  }
  float *out = A.part32 + (int64_t)split * A.T * 3;
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

// Eight waves per SIMD: the register budget (64) still holds the four
// interleaved pair chains of the inner loop.
template <int kTpl>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_far_eq_f32(EqArgs A) {
  const int64_t tile = (int64_t)blockIdx.x * kWavesPerBlock + uniform(threadIdx.x / kWave);
  far_eq_wave<kTpl>(A, tile, blockIdx.y);
}

// FP64 sum of the proxies of the near contact-free spheres of each tile's
// sphere (its near list), one partial slice: the same pair arithmetic as
// the direct sum.
template <int kTpl>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(SMFS_DIRECT_WAVES, 8))) void k_near_f64(
    NearArgs N) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t tile = (int64_t)blockIdx.x * kWavesPerBlock + uniform(threadIdx.x / kWave);
  if (tile >= N.n_tiles) return;
  const int4 tl = N.tiles[tile];
  const int k = uniform(tl.x), t0 = uniform(tl.y), tc = uniform(tl.z);
  if (tc <= 0) return;
  Acc<kTpl> acc;
#pragma unroll
  for (int p = 0; p < kTpl; ++p) {
    const int i = lane + kWave * p;
    const int64_t ti = (int64_t)t0 + (i < tc ? i : 0);
    acc.tx[p] = N.d.tgt[3 * ti];
    acc.ty[p] = N.d.tgt[3 * ti + 1];
    acc.tz[p] = N.d.tgt[3 * ti + 2];
    acc.ax[p] = acc.ay[p] = acc.az[p] = 0.0;
  }
  const int e0 = uniform(N.near_off[k]), e1 = uniform(N.near_off[k + 1]);
  for (int e = e0; e < e1; ++e) {
    const int ks = uniform(N.free_ids[uniform(N.near_idx[e])]);
    const int j0 = uniform((int)N.d.meta[ks].k0[0]);
    const int j1 = j0 + uniform(N.d.meta[ks].kn[0]);
    run_block<kTpl, false>(0, N.d, j0, j1, acc);
  }
#pragma unroll
  for (int p = 0; p < kTpl; ++p) {
    const int i = lane + kWave * p;
    if (i < tc) {
      const int64_t o = 3 * ((int64_t)t0 + i);
      N.out[o] = 0.5 * acc.ax[p];  // the pair functions add twice the velocity
      N.out[o + 1] = 0.5 * acc.ay[p];
      N.out[o + 2] = 0.5 * acc.az[p];
    }
  }
}

// Set-up of the equivalent sources: the Stokeslet matrix K(x, y) without
// the factor 1/(8 pi mu) (3 nx x 3 ny, column-major, ld 3 nx); one thread
// per point pair.
__global__ void k_stokeslet_matrix(const double *__restrict__ x, int32_t nx, const double *__restrict__ y,
                                   int32_t ny, double *__restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nx * ny) return;
  const int i = (int)(idx % nx), j = (int)(idx / nx);
  const double r[3] = {x[3 * i] - y[3 * j], x[3 * i + 1] - y[3 * j + 1], x[3 * i + 2] - y[3 * j + 2]};
  const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
  const double ri = 1.0 / sqrt(r2);
  const int64_t ld = 3 * (int64_t)nx;
  for (int b = 0; b < 3; ++b)
    for (int a = 0; a < 3; ++a)
      out[(3 * (int64_t)j + b) * ld + 3 * i + a] = ((a == b ? 1.0 : 0.0) + r[a] * r[b] / r2) * ri;
}

// A[:, c] /= s[c] for c < cols (column-major, ld rows).
__global__ void k_scale_cols(double *A, int32_t rows, int32_t cols, const double *s) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)rows * cols) return;
  A[idx] /= s[idx / rows];
}

// Packed index of local source jl of sphere m (local order: proxy
// Stokeslets, image Stokeslets, rotlets, dipoles).
__device__ __forceinline__ int64_t packed_index(const SphereMeta &m, int jl) {
  if (jl < m.kn[0]) return m.k0[0] + jl;
  jl -= m.kn[0];
  if (jl < m.kn[1]) return m.k0[1] + jl;
  jl -= m.kn[1];
  if (jl < m.kn[2]) return m.k0[2] + jl;
  return m.k0[3] + (jl - m.kn[2]);
}

__device__ __forceinline__ int block_kind(const SphereMeta &m, int jl) {
  if (jl < m.kn[0] + m.kn[1]) return 0;
  if (jl < m.kn[0] + m.kn[1] + m.kn[2]) return 1;
  return 2;
}

// ---------------------------------------------------------------------------
// Pseudo-inverse apply: one wave per output row, a dot product of a
// contiguous factor row with a short vector.

// A factor entry read once per product: a non-temporal load, so that the
// streamed factor does not evict the vector slice that the waves of the
// same sphere share in the cache.
__device__ __forceinline__ double stream_load(const double *p) {
  return __builtin_nontemporal_load(p);
}

// One wave per row j of U^T: sbuf[s0 + j] = (U_k^T mu)_j / sigma_j.
__device__ __forceinline__ void pinv_u_row(const RowTask *__restrict__ tasks, int64_t t,
                                           const SphereMeta *__restrict__ meta,
                                           const FactorSlot *__restrict__ fs,
                                           const double *__restrict__ fac,
                                           const double *__restrict__ mu, double *__restrict__ sbuf) {
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
    a0 = fma(stream_load(col + i), x[i], a0);
    a1 = fma(stream_load(col + i + kWave), x[i + kWave], a1);
    a2 = fma(stream_load(col + i + 2 * kWave), x[i + 2 * kWave], a2);
    a3 = fma(stream_load(col + i + 3 * kWave), x[i + 3 * kWave], a3);
  }
  for (; i < rows; i += kWave) a0 = fma(stream_load(col + i), x[i], a0);
  const double s = wave_sum((a0 + a1) + (a2 + a3));
  if (lane == 0) sbuf[m.s0 + j] = s / fac[f.sig_off + j];
}

// One wave per row r of V: lam[packed(r)] = (V_k s)_r, dipoles times dscale.
__device__ __forceinline__ void pinv_v_row(const RowTask *__restrict__ tasks, int64_t t,
                                           const SphereMeta *__restrict__ meta,
                                           const FactorSlot *__restrict__ fs,
                                           const double *__restrict__ fac,
                                           const double *__restrict__ sbuf,
                                           double *__restrict__ lam, double dscale) {
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
    a0 = fma(stream_load(row + i), x[i], a0);
    a1 = fma(stream_load(row + i + kWave), x[i + kWave], a1);
    a2 = fma(stream_load(row + i + 2 * kWave), x[i + 2 * kWave], a2);
    a3 = fma(stream_load(row + i + 3 * kWave), x[i + 3 * kWave], a3);
  }
  for (; i < rank; i += kWave) a0 = fma(stream_load(row + i), x[i], a0);
  const double s = wave_sum((a0 + a1) + (a2 + a3));
  if (lane == 0) {
    const int jl = r / 3, c = r - 3 * (r / 3);
    const bool dip = jl >= m.kn[0] + m.kn[1] + m.kn[2];
    lam[3 * packed_index(m, jl) + c] = dip ? s * dscale : s;
  }
}

// kPinvRows consecutive rows j.. of one sphere per wave: the slice of mu is
// loaded once for all of them (same summation order per row as
// pinv_u_row, so the results are identical).  Groups that straddle a sphere
// fall back to one row at a time.
constexpr int kPinvRows = 2;   // 4 measured no faster

__global__ __launch_bounds__(kBlock) void k_pinv_u(const RowTask *__restrict__ tasks, int64_t n,
                                                   const SphereMeta *__restrict__ meta,
                                                   const FactorSlot *__restrict__ fs,
                                                   const double *__restrict__ fac,
                                                   const double *__restrict__ mu,
                                                   double *__restrict__ sbuf) {
  const int64_t t = kPinvRows * ((int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave);
  if (t >= n) return;
  const int k0 = uniform(tasks[t].sphere), j0 = uniform(tasks[t].row);
  bool fused = t + kPinvRows <= n;
  if (fused) {
    const RowTask last = tasks[t + kPinvRows - 1];
    fused = uniform(last.sphere) == k0 && uniform(last.row) == j0 + kPinvRows - 1;
  }
  if (!fused) {
    for (int r = 0; r < kPinvRows && t + r < n; ++r) pinv_u_row(tasks, t + r, meta, fs, fac, mu, sbuf);
    return;
  }
  const int lane = threadIdx.x & (kWave - 1);
  const SphereMeta &m = meta[k0];
  const FactorSlot &f = fs[m.fid];
  const int rows = f.rows;
  const double *c0 = fac + f.u_off + (int64_t)j0 * rows;
  const double *x = mu + 3 * m.t0;
  double a[kPinvRows][4];
#pragma unroll
  for (int r = 0; r < kPinvRows; ++r) a[r][0] = a[r][1] = a[r][2] = a[r][3] = 0.0;
  int i = lane;
  for (; i + 3 * kWave < rows; i += 4 * kWave) {
    double xv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) xv[u] = x[i + u * kWave];
#pragma unroll
    for (int r = 0; r < kPinvRows; ++r)
#pragma unroll
      for (int u = 0; u < 4; ++u)
        a[r][u] = fma(stream_load(c0 + (int64_t)r * rows + i + u * kWave), xv[u], a[r][u]);
  }
  for (; i < rows; i += kWave) {
    const double xi = x[i];
#pragma unroll
    for (int r = 0; r < kPinvRows; ++r) a[r][0] = fma(stream_load(c0 + (int64_t)r * rows + i), xi, a[r][0]);
  }
#pragma unroll
  for (int r = 0; r < kPinvRows; ++r) {
    // rows whose tasks were checked: j0 .. j0 + kPinvRows - 1 of sphere k0
    const double sr = wave_sum((a[r][0] + a[r][1]) + (a[r][2] + a[r][3]));
    if (lane == 0) sbuf[m.s0 + j0 + r] = sr / fac[f.sig_off + j0 + r];
  }
}

__global__ __launch_bounds__(kBlock) void k_pinv_v(const RowTask *__restrict__ tasks, int64_t n,
                                                   const SphereMeta *__restrict__ meta,
                                                   const FactorSlot *__restrict__ fs,
                                                   const double *__restrict__ fac,
                                                   const double *__restrict__ sbuf,
                                                   double *__restrict__ lam, double dscale) {
  const int64_t t = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  if (t >= n) return;
  pinv_v_row(tasks, t, meta, fs, fac, sbuf, lam, dscale);
}


__global__ void k_to_f32(int64_t n, const double *__restrict__ x, float *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}

// ---------------------------------------------------------------------------
// Right-hand side, forces/torques, residual statistics.

// Boundary data of eq. (bc) at point x of sphere k: v + omega x (x - c) minus
// the background flow U + L x (when bg.on); rbm == NULL means rest.
__device__ __forceinline__ void boundary_data(const double *__restrict__ x,
                                              const SphereMeta &m, const double *__restrict__ rbm,
                                              int k, const BgFlow &bg, double (&w)[3]) {
  w[0] = w[1] = w[2] = 0.0;
  if (rbm) {
    const double *v = rbm + 6 * (int64_t)k;
    const double rx = x[0] - m.c[0], ry = x[1] - m.c[1], rz = x[2] - m.c[2];
    w[0] = v[0] + v[4] * rz - v[5] * ry;
    w[1] = v[1] + v[5] * rx - v[3] * rz;
    w[2] = v[2] + v[3] * ry - v[4] * rx;
  }
  if (bg.on) {
#pragma unroll
    for (int q = 0; q < 3; ++q)
      w[q] -= bg.U[q] + bg.L[3 * q] * x[0] + bg.L[3 * q + 1] * x[1] + bg.L[3 * q + 2] * x[2];
  }
}

// y = alpha W u_bc + (beta != 0 ? beta y : 0) at the nodes, u_bc the
// boundary data above.
__global__ void k_rigid(int64_t T, const double *__restrict__ tgt, const int32_t *__restrict__ tsph,
                        const double *__restrict__ sw, const SphereMeta *__restrict__ meta,
                        const double *__restrict__ rbm, BgFlow bg, double alpha, double beta,
                        double *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T) return;
  const int k = tsph[i];
  double w[3];
  boundary_data(tgt + 3 * i, meta[k], rbm, k, bg, w);
  const double s = alpha * sw[i];
  const double u0 = s * w[0];
  const double u1 = s * w[1];
  const double u2 = s * w[2];
  if (beta != 0.0) {
    y[3 * i] = fma(beta, y[3 * i], u0);
    y[3 * i + 1] = fma(beta, y[3 * i + 1], u1);
    y[3 * i + 2] = fma(beta, y[3 * i + 2], u2);
  } else {
    y[3 * i] = u0;
    y[3 * i + 1] = u1;
    y[3 * i + 2] = u2;
  }
}

// y[6k + q] = x[6k + q] * (q < 3 ? sF : sT)
__global__ void k_scale_ft(int32_t P, const double *__restrict__ x, double sF, double sT,
                           double *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 6 * (int64_t)P) return;
  y[i] = x[i] * ((i % 6) < 3 ? sF : sT);
}

__global__ __launch_bounds__(kBlock) void k_force_torque(const SphereMeta *__restrict__ meta,
                                                         const double *__restrict__ src,
                                                         const double *__restrict__ lam,
                                                         double *__restrict__ ft, double sF,
                                                         double sT) {
  __shared__ double sh[6][kWavesPerBlock];
  const int k = blockIdx.x;
  const SphereMeta &m = meta[k];
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int j = threadIdx.x; j < m.kn[0] + m.kn[1]; j += kBlock) {
    const int64_t p = j < m.kn[0] ? m.k0[0] + j : m.k0[1] + (j - m.kn[0]);
    const double f0 = lam[3 * p], f1 = lam[3 * p + 1], f2 = lam[3 * p + 2];
    const double y0 = src[3 * p] - m.c[0], y1 = src[3 * p + 1] - m.c[1], y2 = src[3 * p + 2] - m.c[2];
    v[0] += f0;
    v[1] += f1;
    v[2] += f2;
    v[3] += y1 * f2 - y2 * f1;
    v[4] += y2 * f0 - y0 * f2;
    v[5] += y0 * f1 - y1 * f0;
  }
  for (int j = threadIdx.x; j < m.kn[2]; j += kBlock) {
    const int64_t p = m.k0[2] + j;
    v[3] += lam[3 * p];
    v[4] += lam[3 * p + 1];
    v[5] += lam[3 * p + 2];
  }
  block_sum<6>(v, sh);
  if (threadIdx.x < 6) ft[6 * k + threadIdx.x] = v[threadIdx.x] * (threadIdx.x < 3 ? sF : sT);
}

__global__ __launch_bounds__(1024) void k_residual_stats(int64_t n, const double *__restrict__ pts,
                                                         const int32_t *__restrict__ sph,
                                                         const SphereMeta *__restrict__ meta,
                                                         const double *__restrict__ rbm,
                                                         BgFlow bg,
                                                         const double *__restrict__ u,
                                                         double floor_rel, double *out) {
  __shared__ double sh[16];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  auto ubc = [&](int64_t i, double (&w)[3]) {
    const int k = sph[i];
    boundary_data(pts + 3 * i, meta[k], rbm, k, bg, w);
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
  const int kind = block_kind(m, (int)jl);
  const int64_t p = packed_index(m, (int)jl);
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

__global__ void k_mdot_final(int32_t nv, const double *__restrict__ part, int32_t nchunks,
                             double *__restrict__ h, int acc) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nv) return;
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += part[(int64_t)j * nchunks + c];
  h[j] = acc ? h[j] + s : s;
}

// sum_j V[j][i] c[j] for element i of nv basis vectors (stride ld): eight
// loads in flight per step and four partial sums, so that the loop is
// bound by HBM bandwidth rather than by one load latency per vector.
__device__ __forceinline__ double basis_row_dot(const double *__restrict__ V, int64_t ld, int nv,
                                                const double *__restrict__ c, int64_t i) {
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  int j = 0;
  for (; j + 7 < nv; j += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = V[(int64_t)(j + u) * ld + i];
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u & 3] = fma(v[u], c[j + u], s[u & 3]);
  }
  for (; j < nv; ++j) s[0] = fma(V[(int64_t)j * ld + i], c[j], s[0]);
  return (s[0] + s[1]) + (s[2] + s[3]);
}

__global__ void k_combine(const double *__restrict__ V, int64_t ld, int32_t nv,
                          const double *__restrict__ cf, double *__restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  x[i] += basis_row_dot(V, ld, nv, cf, i);
}

// Delayed classical Gram-Schmidt (one pass of dot products and one pass of
// updates per Arnoldi step; the second Gram-Schmidt pass of the previous
// vector rides along with the first pass of the new one).
// part[(r * nv + j) * nchunks + c] = chunk c of V[j] . (r ? b : a)
constexpr int kDot2Vecs = 8;    // basis vectors per block of the two-vector dot products (16 measured 2.6x slower)

__global__ __launch_bounds__(kBlock) void k_mdot2(const double *__restrict__ V, int64_t ld,
                                                  int32_t nv, const double *__restrict__ a,
                                                  const double *__restrict__ b, int64_t n,
                                                  int64_t chunk, double *__restrict__ part,
                                                  int32_t nchunks) {
  __shared__ double sh[2 * kDot2Vecs][kWavesPerBlock];
  const int c = blockIdx.x;
  const int j0 = blockIdx.y * kDot2Vecs;
  const int64_t e0 = (int64_t)c * chunk, e1 = min(n, e0 + chunk);
  double acc[2 * kDot2Vecs];
#pragma unroll
  for (int q = 0; q < 2 * kDot2Vecs; ++q) acc[q] = 0.0;
  for (int64_t i = e0 + threadIdx.x; i < e1; i += kBlock) {
    const double ai = a[i], bi = b[i];
#pragma unroll
    for (int q = 0; q < kDot2Vecs; ++q)
      if (j0 + q < nv) {
        const double v = stream_load(V + (int64_t)(j0 + q) * ld + i);
        acc[q] = fma(v, ai, acc[q]);
        acc[kDot2Vecs + q] = fma(v, bi, acc[kDot2Vecs + q]);
      }
  }
  block_sum<2 * kDot2Vecs>(acc, sh);
  if (threadIdx.x < 2 * kDot2Vecs) {
    const int q = threadIdx.x % kDot2Vecs, r = threadIdx.x / kDot2Vecs;
    if (j0 + q < nv) part[((int64_t)r * nv + j0 + q) * nchunks + c] = acc[threadIdx.x];
  }
}

// The scalars of a delayed Gram-Schmidt step from the dot products
// h = [V^T q (nv) | V^T w (nv)] with nv = j + 1 (one thread, the sums in
// index order): nu = sqrt(h_j - sum_{i<j} h_i^2) (1 for j = 0, 0 if the
// difference is not positive), gam = (h_{nv+j} - sum_{i<j} h_i h_{nv+i}) / nu;
// out = [1/nu, gam, nu].
__global__ void k_dcgs_coeffs(const double *__restrict__ h, int32_t j, double *__restrict__ out) {
  if (threadIdx.x != 0) return;
  const int nv = j + 1;
  double nu = 1.0;
  if (j > 0) {
    double ss = 0.0;
    for (int i = 0; i < j; ++i) ss += h[i] * h[i];
    const double nu2 = h[j] - ss;
    nu = nu2 > 0.0 ? sqrt(nu2) : 0.0;
  }
  double sz = 0.0;
  for (int i = 0; i < j; ++i) sz += h[i] * h[nv + i];
  out[0] = 1.0 / nu;
  out[1] = (h[nv + j] - sz) / nu;
  out[2] = nu;
}

// q <- (q - V cs) / nu ;  w <- (w - V cz - q gam) / nu over V[0..nb), one
// read of the basis (coeffs = [1/nu, gam] on the device); part[block] = sum
// of the new w^2 over the block.
__global__ __launch_bounds__(kBlock) void k_dcgs_update(const double *__restrict__ V, int64_t ld,
                                                        int32_t nb, const double *__restrict__ cs,
                                                        const double *__restrict__ cz,
                                                        double *__restrict__ q,
                                                        double *__restrict__ w,
                                                        const double *__restrict__ coeffs,
                                                        int64_t n, double *__restrict__ part) {
  __shared__ double sh[1][kWavesPerBlock];
  const double inv_nu = coeffs[0], gam = coeffs[1];
  double acc[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    double s1[2] = {0.0, 0.0}, s2[2] = {0.0, 0.0};
    int j = 0;
    for (; j + 7 < nb; j += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = stream_load(V + (int64_t)(j + u) * ld + i);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        s1[u & 1] = fma(v[u], cs[j + u], s1[u & 1]);
        s2[u & 1] = fma(v[u], cz[j + u], s2[u & 1]);
      }
    }
    for (; j < nb; ++j) {
      const double v = stream_load(V + (int64_t)j * ld + i);
      s1[0] = fma(v, cs[j], s1[0]);
      s2[0] = fma(v, cz[j], s2[0]);
    }
    const double qt = (q[i] - (s1[0] + s1[1])) * inv_nu;
    const double p = ((w[i] - (s2[0] + s2[1])) - qt * gam) * inv_nu;
    q[i] = qt;
    w[i] = p;
    acc[0] = fma(p, p, acc[0]);
  }
  block_sum<1>(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
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

// One block: beta[0] = out[0] = sqrt(sum of the nchunks partial sums).
__global__ __launch_bounds__(kBlock) void k_sqrt_final(const double *__restrict__ part,
                                                       int32_t nchunks, double *beta, double *out) {
  __shared__ double sh[1][kWavesPerBlock];
  double acc[1] = {0.0};
  for (int c = threadIdx.x; c < nchunks; c += kBlock) acc[0] += part[c];
  block_sum<1>(acc, sh);
  if (threadIdx.x == 0) {
    const double s = sqrt(acc[0]);
    if (beta) beta[0] = s;
    if (out) out[0] = s;
  }
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

__host__ __device__ inline int64_t chunk_len(int64_t n, int32_t nchunks) { return (n + nchunks - 1) / nchunks; }

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
    hipLaunchKernelGGL((k_direct_f64<kDirectTpl, false>), grid, dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((k_direct_f64<kDirectTpl, true>), grid, dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_far_f32(const Far32Args &a, hipStream_t s) {
  if (a.n_tiles == 0 || a.n_splits == 0) return hipSuccess;
  dim3 grid((unsigned)((a.n_tiles + kWavesPerBlock - 1) / kWavesPerBlock), (unsigned)a.n_splits);
  hipLaunchKernelGGL((k_far_f32<kDirectTpl>), grid, dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_eq_strengths(const double *E, int32_t rows, int32_t cols, const double *lam,
                               const SphereMeta *meta, const int32_t *free_ids, int32_t n_free, float *q32,
                               hipStream_t s) {
  if (n_free <= 0 || rows <= 0) return hipSuccess;
  dim3 grid((unsigned)((rows + 255) / 256), (unsigned)((n_free + 3) / 4));
  hipLaunchKernelGGL(k_eq_strengths, grid, dim3(256), 0, s, E, rows, cols, lam, meta, free_ids, n_free, q32);
  return hipGetLastError();
}

hipError_t launch_far_eq_f32(const EqArgs &a, hipStream_t s) {
  if (a.n_tiles == 0 || a.n_splits == 0) return hipSuccess;
  dim3 grid((unsigned)((a.n_tiles + kWavesPerBlock - 1) / kWavesPerBlock), (unsigned)a.n_splits);
  hipLaunchKernelGGL((k_far_eq_f32<kDirectTpl>), grid, dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_near_f64(const NearArgs &a, hipStream_t s) {
  if (a.n_tiles == 0) return hipSuccess;
  dim3 grid((unsigned)((a.n_tiles + kWavesPerBlock - 1) / kWavesPerBlock));
  hipLaunchKernelGGL((k_near_f64<kDirectTpl>), grid, dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_stokeslet_matrix(const double *x, int32_t nx, const double *y, int32_t ny, double *out,
                                   hipStream_t s) {
  const int64_t n = (int64_t)nx * ny;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_stokeslet_matrix, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, nx, y, ny, out);
  return hipGetLastError();
}

hipError_t launch_scale_cols(double *A, int32_t rows, int32_t cols, const double *sv, hipStream_t s) {
  const int64_t n = (int64_t)rows * cols;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_cols, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, rows, cols, sv);
  return hipGetLastError();
}

hipError_t launch_reduce_epilogue(int64_t n3, int32_t ns, const double *part, int32_t ns32,
                                  const float *part32, const double *base, const double *sw,
                                  double c0, double *y, hipStream_t s) {
  if (n3 == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_epilogue, dim3(blocks_for(n3)), dim3(kBlock), 0, s, n3, ns, part,
                     ns32, part32, base, sw, c0, y);
  return hipGetLastError();
}


hipError_t launch_to_f32(int64_t n, const double *x, float *y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, x, y);
  return hipGetLastError();
}

hipError_t launch_pinv_u(const RowTask *tasks, int64_t n, const SphereMeta *meta,
                         const FactorSlot *fs, const double *fac, const double *mu, double *sbuf,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pinv_u, dim3(blocks_for((n + kPinvRows - 1) / kPinvRows, kWavesPerBlock)),
                     dim3(kBlock), 0, s, tasks, n, meta, fs, fac, mu, sbuf);
  return hipGetLastError();
}

hipError_t launch_pinv_v(const RowTask *tasks, int64_t n, const SphereMeta *meta,
                         const FactorSlot *fs, const double *fac, const double *sbuf, double *lam,
                         double dscale, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pinv_v, dim3(blocks_for(n, kWavesPerBlock)), dim3(kBlock), 0, s, tasks, n,
                     meta, fs, fac, sbuf, lam, dscale);
  return hipGetLastError();
}

namespace {
BgFlow bg_or_rest(const BgFlow *bg) {
  BgFlow r{};
  if (bg && bg->on) r = *bg;
  return r;
}
}  // namespace

hipError_t launch_rigid(int64_t T, const double *tgt, const int32_t *tsph, const double *sw,
                        const SphereMeta *meta, const double *rbm, double alpha, double beta,
                        double *y, hipStream_t s, const BgFlow *bg) {
  if (T == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rigid, dim3(blocks_for(T)), dim3(kBlock), 0, s, T, tgt, tsph, sw, meta, rbm,
                     bg_or_rest(bg), alpha, beta, y);
  return hipGetLastError();
}

hipError_t launch_rhs(int64_t T, const double *tgt, const int32_t *tsph, const double *sw,
                      const SphereMeta *meta, const double *rbm, double *b, hipStream_t s,
                      const BgFlow *bg) {
  return launch_rigid(T, tgt, tsph, sw, meta, rbm, 1.0, 0.0, b, s, bg);
}

hipError_t launch_force_torque(int32_t P, const SphereMeta *meta, const double *src,
                               const double *lam, double *ft, hipStream_t s, double sF, double sT) {
  if (P == 0) return hipSuccess;
  hipLaunchKernelGGL(k_force_torque, dim3(P), dim3(kBlock), 0, s, meta, src, lam, ft, sF, sT);
  return hipGetLastError();
}

hipError_t launch_scale_ft(int32_t P, const double *x, double sF, double sT, double *y,
                           hipStream_t s) {
  if (P == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_ft, dim3(blocks_for(6 * (int64_t)P)), dim3(kBlock), 0, s, P, x, sF, sT, y);
  return hipGetLastError();
}

hipError_t launch_residual_stats(int64_t n, const double *pts, const int32_t *sph,
                                 const SphereMeta *meta, const double *rbm, const double *u,
                                 double floor_rel, double *out, hipStream_t s, const BgFlow *bg) {
  hipLaunchKernelGGL(k_residual_stats, dim3(1), dim3(1024), 0, s, n, pts, sph, meta, rbm,
                     bg_or_rest(bg), u, floor_rel, out);
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
  hipLaunchKernelGGL(k_sqrt_final, dim3(1), dim3(kBlock), 0, s, part, nchunks, (double *)nullptr, out);
  return hipGetLastError();
}

hipError_t launch_mdot2(const double *V, int64_t ld, int32_t nv, const double *a, const double *b,
                        int64_t n, double *part, int32_t nchunks, double *out, hipStream_t s) {
  if (nv <= 0) return hipSuccess;
  const int64_t chunk = chunk_len(n, nchunks);
  dim3 grid((unsigned)nchunks, (unsigned)((nv + kDot2Vecs - 1) / kDot2Vecs));
  hipLaunchKernelGGL(k_mdot2, grid, dim3(kBlock), 0, s, V, ld, nv, a, b, n, chunk, part, nchunks);
  hipLaunchKernelGGL(k_mdot_final, dim3(blocks_for(2 * nv)), dim3(kBlock), 0, s, 2 * nv, part, nchunks,
                     out, 0);
  return hipGetLastError();
}

hipError_t launch_dcgs_coeffs(const double *h, int32_t j, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_dcgs_coeffs, dim3(1), dim3(kWave), 0, s, h, j, out);
  return hipGetLastError();
}

hipError_t launch_dcgs_update(const double *V, int64_t ld, int32_t nb, const double *cs,
                              const double *cz, double *q, double *w, const double *coeffs, int64_t n,
                              double *part, int32_t nparts, double *norm, hipStream_t s) {
  const unsigned g = (unsigned)std::min<int64_t>(nparts, blocks_for(n));
  hipLaunchKernelGGL(k_dcgs_update, dim3(g), dim3(kBlock), 0, s, V, ld, nb, cs, cz, q, w, coeffs, n,
                     part);
  hipLaunchKernelGGL(k_sqrt_final, dim3(1), dim3(kBlock), 0, s, part, (int32_t)g, norm, nullptr);
  hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, s, w, n, norm);
  return hipGetLastError();
}

hipError_t launch_norm_scale(double *w, int64_t n, double *part, int32_t nchunks, double *beta,
                             double *out, hipStream_t s) {
  const int64_t chunk = chunk_len(n, nchunks);
  hipLaunchKernelGGL(k_sumsq, dim3(nchunks), dim3(kBlock), 0, s, w, n, chunk, part);
  hipLaunchKernelGGL(k_sqrt_final, dim3(1), dim3(kBlock), 0, s, part, nchunks, beta, out);
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

// ===========================================================================
// Many right-hand sides (block product).  Vectors of the block are stored
// one after another (stride ld); strengths of the block are source-major,
// lamb[(p * nrhs + q) * 3 + c], so one source's strengths for a run of
// right-hand sides are contiguous.

namespace smfs {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Tasks of the block pseudo-inverse apply are (sphere, first row of a
// 32-row tile); blockIdx.y picks the 32-wide tile of right-hand sides.
//
// One 32 x 32 output tile per wave of C = A B (A row i contiguous over k,
// B column j contiguous over k) on v_mfma_f64_16x16x4f64.  Lane l supplies
// A[i0 + l%16][k] and B[k][j0 + l%16] for the k-slot l/16 of a step, and
// after the sum holds C[i0 + 4v + l/16][j0 + l%16] in register v.  Each
// lane loads four consecutive k per 16-wide k chunk and the four steps take
// k = kc + 4 (l/16) + s, which covers the chunk.
struct TileTN {
  f64x4 acc[2][2];
};

__device__ __forceinline__ void mfma_tile_tn(const double *const arow[2], const bool aok[2],
                                             const double *const bcol[2], const bool bok[2],
                                             int64_t K, TileTN &t) {
  const int lane = threadIdx.x & 63, g = lane >> 4;
#pragma unroll
  for (int ia = 0; ia < 2; ++ia)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) t.acc[ia][jb] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int64_t kc = 0; kc < K; kc += 16) {
    double a[2][4], b[2][4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t k = kc + 4 * g + s;
      const bool kin = k < K;
#pragma unroll
      for (int ia = 0; ia < 2; ++ia) a[ia][s] = (aok[ia] && kin) ? arow[ia][k] : 0.0;
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) b[jb][s] = (bok[jb] && kin) ? bcol[jb][k] : 0.0;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int ia = 0; ia < 2; ++ia)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
          t.acc[ia][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ia][s], b[jb][s], t.acc[ia][jb], 0, 0, 0);
  }
}

// One 64 x 64 tile of C = A B per workgroup of four waves, each wave a
// 32 x 32 quarter as in mfma_tile_tn.  A rows (rowsA of them, stride lda)
// and B columns (colsB, stride ldb) are contiguous over k; chunks of 16 k of
// both are staged through LDS, so every element is read from memory once
// per workgroup (the factor once per 64 right-hand sides, the vectors once
// per 64 rows), and double-buffered: the global loads of the next chunk are
// in flight while the MFMAs run on this one.  The k order of every sum is
// that of mfma_tile_tn.
constexpr int kGT = 64, kGK = 16, kGP = kGK + 2;   // tile, k chunk, padded LDS row
struct GemmLds {
  double a[2][kGT][kGP];
  double b[2][kGT][kGP];
};

__device__ __forceinline__ void gemm_tile_lds(const double *__restrict__ A, int64_t lda, int rowsA,
                                              const double *__restrict__ B, int64_t ldb, int colsB, int64_t K,
                                              GemmLds &sh, TileTN &t) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int lr = tid >> 2, lk = (tid & 3) * 4;    // this thread's staging row and k offset
  const bool aok = lr < rowsA, bok = lr < colsB;
  const double *ap = A + (int64_t)(aok ? lr : 0) * lda;
  const double *bp = B + (int64_t)(bok ? lr : 0) * ldb;
#pragma unroll
  for (int ia = 0; ia < 2; ++ia)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) t.acc[ia][jb] = f64x4{0.0, 0.0, 0.0, 0.0};
  double ra[4], rb[4];
  auto fetch = [&](int64_t kc) {
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      const int64_t k = kc + lk + s2;
      ra[s2] = (aok && k < K) ? ap[k] : 0.0;
      rb[s2] = (bok && k < K) ? bp[k] : 0.0;
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      sh.a[buf][lr][lk + s2] = ra[s2];
      sh.b[buf][lr][lk + s2] = rb[s2];
    }
  };
  const int64_t nch = (K + kGK - 1) / kGK;
  if (nch > 0) {
    fetch(0);
    stage(0);
  }
  __syncthreads();
  for (int64_t c = 0; c < nch; ++c) {
    const int cur = (int)(c & 1);
    if (c + 1 < nch) fetch((c + 1) * kGK);
    double a[2][4], b[2][4];
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
#pragma unroll
      for (int ia = 0; ia < 2; ++ia) a[ia][s2] = sh.a[cur][wr + 16 * ia + li][4 * g + s2];
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) b[jb][s2] = sh.b[cur][wc + 16 * jb + li][4 * g + s2];
    }
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
      for (int ia = 0; ia < 2; ++ia)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
          t.acc[ia][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ia][s2], b[jb][s2], t.acc[ia][jb], 0, 0, 0);
    if (c + 1 < nch) stage(cur ^ 1);
    __syncthreads();
  }
}

// S[q][s0 + r] = (U_k^T mu_q)_r / sigma_r for the rows r of the tile
// (tasks: sphere and first row of a 64-row tile; blockIdx.y: 64 right-hand
// sides).
__global__ __launch_bounds__(kBlock) void k_pinv_block_u(const int4 *__restrict__ tasks, int64_t n,
                                                         const SphereMeta *__restrict__ meta,
                                                         const FactorSlot *__restrict__ fs,
                                                         const double *__restrict__ fac,
                                                         const double *__restrict__ mu, int64_t ldmu,
                                                         int32_t nrhs, double *__restrict__ S,
                                                         int64_t lds) {
  __shared__ GemmLds sh;
  const int64_t t = blockIdx.x;
  if (t >= n) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int4 tk = tasks[t];
  const int k = tk.x, r0 = tk.y, q0 = blockIdx.y * kGT;
  const SphereMeta &m = meta[k];
  const FactorSlot &f = fs[m.fid];
  const int rank = m.rank;
  TileTN tile;
  gemm_tile_lds(fac + f.u_off + (int64_t)r0 * f.rows, f.rows, rank - r0, mu + (int64_t)q0 * ldmu + 3 * m.t0, ldmu,
                nrhs - q0, f.rows, sh, tile);
  const double *sig = fac + f.sig_off;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  for (int ia = 0; ia < 2; ++ia)
    for (int jb = 0; jb < 2; ++jb)
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + wr + 16 * ia + 4 * v + (lane >> 4), q = q0 + wc + 16 * jb + (lane & 15);
        if (r < rank && q < nrhs) S[(int64_t)q * lds + m.s0 + r] = tile.acc[ia][jb][v] / sig[r];
      }
}

// lamb[packed(row)][q] = (V_k S_q)_row, dipoles multiplied by dscale.
__global__ __launch_bounds__(kBlock) void k_pinv_block_v(const int4 *__restrict__ tasks, int64_t n,
                                                         const SphereMeta *__restrict__ meta,
                                                         const FactorSlot *__restrict__ fs,
                                                         const double *__restrict__ fac,
                                                         const double *__restrict__ S, int64_t lds,
                                                         int32_t nrhs, double *__restrict__ lamb,
                                                         double dscale) {
  __shared__ GemmLds sh;
  const int64_t t = blockIdx.x;
  if (t >= n) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int4 tk = tasks[t];
  const int k = tk.x, r0 = tk.y, q0 = blockIdx.y * kGT;
  const SphereMeta &m = meta[k];
  const FactorSlot &f = fs[m.fid];
  const int rows = f.cols;
  TileTN tile;
  gemm_tile_lds(fac + f.vt_off + (int64_t)r0 * f.cols, f.cols, rows - r0, S + (int64_t)q0 * lds + m.s0, lds,
                nrhs - q0, m.rank, sh, tile);
  const int nd0 = m.kn[0] + m.kn[1] + m.kn[2];
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  for (int ia = 0; ia < 2; ++ia)
    for (int jb = 0; jb < 2; ++jb)
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + wr + 16 * ia + 4 * v + (lane >> 4), q = q0 + wc + 16 * jb + (lane & 15);
        if (r < rows && q < nrhs) {
          const int jl = r / 3, c = r - 3 * (r / 3);
          const double val = tile.acc[ia][jb][v];
          lamb[(packed_index(m, jl) * nrhs + q) * 3 + c] = jl >= nd0 ? val * dscale : val;
        }
      }
}

// Block direct sum: as k_direct_f64 but every pair serves a run of kRun
// right-hand sides (blockIdx.z picks the run); the geometry (r, 1/|r|) is
// computed once per pair and run.
template <int kTpl, int kRun>
struct AccB {
  double tx[kTpl], ty[kTpl], tz[kTpl];
  double a[kTpl][kRun][3];
};

// As the pair functions of the single-vector sum, every pair adds twice its
// velocity (Y = 2/|r| from rsq2_f64; the Stokeslet's r.f is formed with
// g = f/4), and the tile's sums are halved once when stored.  Source indices
// fit in 32 bits and the bounds are wave-uniform, so the loop test runs on
// the scalar unit.
template <int kTpl, int kRun, int kKind>
__device__ __forceinline__ void run_sources_block(const double *__restrict__ src_,
                                                  const double *__restrict__ lamb_, int32_t nrhs,
                                                  int q0, int64_t j0_, int64_t j1_,
                                                  AccB<kTpl, kRun> &A) {
  const ConstPtr src = (ConstPtr)src_, lamb = (ConstPtr)lamb_;
  const int j1 = uniform((int)j1_);
  for (int j = uniform((int)j0_); j < j1; ++j) {
    const ConstPtr ps = src + 3 * j;
    const ConstPtr pf = lamb + ((int64_t)j * nrhs + q0) * 3;
    const double sx = ps[0], sy = ps[1], sz = ps[2];
    double f[kRun][3], g[kRun][3];
#pragma unroll
    for (int q = 0; q < kRun; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        f[q][c] = pf[3 * q + c];
        g[q][c] = quarter(f[q][c]);
      }
#pragma unroll
    for (int p = 0; p < kTpl; ++p) {
      const double rx = A.tx[p] - sx, ry = A.ty[p] - sy, rz = A.tz[p] - sz;
      const double r2 = fma(rx, rx, fma(ry, ry, rz * rz));
      const double Y = rsq2_f64(r2);
      const double Y2 = Y * Y;
      if (kKind == 0) {
#pragma unroll
        for (int q = 0; q < kRun; ++q) {
          const double rg = fma(rx, g[q][0], fma(ry, g[q][1], rz * g[q][2]));
          const double t = rg * Y2;
          A.a[p][q][0] = fma(fma(rx, t, f[q][0]), Y, A.a[p][q][0]);
          A.a[p][q][1] = fma(fma(ry, t, f[q][1]), Y, A.a[p][q][1]);
          A.a[p][q][2] = fma(fma(rz, t, f[q][2]), Y, A.a[p][q][2]);
        }
      } else if (kKind == 1) {
        const double c = (0.25 * Y) * Y2;                 // 2/|r|^3
#pragma unroll
        for (int q = 0; q < kRun; ++q) {
          A.a[p][q][0] = fma(c, fma(f[q][1], rz, -f[q][2] * ry), A.a[p][q][0]);
          A.a[p][q][1] = fma(c, fma(f[q][2], rx, -f[q][0] * rz), A.a[p][q][1]);
          A.a[p][q][2] = fma(c, fma(f[q][0], ry, -f[q][1] * rx), A.a[p][q][2]);
        }
      } else {
        const double c3 = 0.25 * (Y2 * Y);               // 2/|r|^3
        const double c5 = (0.75 * c3) * Y2;              // 6/|r|^5
#pragma unroll
        for (int q = 0; q < kRun; ++q) {
          const double bb = fma(rx, f[q][0], fma(ry, f[q][1], rz * f[q][2])) * c5;
          A.a[p][q][0] = fma(-f[q][0], c3, fma(rx, bb, A.a[p][q][0]));
          A.a[p][q][1] = fma(-f[q][1], c3, fma(ry, bb, A.a[p][q][1]));
          A.a[p][q][2] = fma(-f[q][2], c3, fma(rz, bb, A.a[p][q][2]));
        }
      }
    }
  }
}

template <int kTpl, int kRun>
__device__ __forceinline__ void run_block_b(int block, const BlockDirectArgs &A, int q0, int64_t j0,
                                            int64_t j1, AccB<kTpl, kRun> &acc) {
  if (j0 >= j1) return;
  if (block <= 1) run_sources_block<kTpl, kRun, 0>(A.src, A.lamb, A.nrhs, q0, j0, j1, acc);
  else if (block == 2) run_sources_block<kTpl, kRun, 1>(A.src, A.lamb, A.nrhs, q0, j0, j1, acc);
  else run_sources_block<kTpl, kRun, 2>(A.src, A.lamb, A.nrhs, q0, j0, j1, acc);
}

template <int kTpl, int kRun>
__global__ __launch_bounds__(kBlock) void k_direct_block(BlockDirectArgs A) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t tile = (int64_t)blockIdx.x * kWavesPerBlock + uniform(threadIdx.x / kWave);
  if (tile >= A.n_tiles) return;
  const int4 tl = A.tiles[tile];
  const int k = uniform(tl.x), t0 = uniform(tl.y), tc = uniform(tl.z);
  const int q0 = blockIdx.z * kRun;
  AccB<kTpl, kRun> acc;
#pragma unroll
  for (int p = 0; p < kTpl; ++p) {
    const int i = lane + kWave * p;
    const int64_t ti = (int64_t)t0 + (i < tc ? i : 0);
    acc.tx[p] = A.tgt[3 * ti];
    acc.ty[p] = A.tgt[3 * ti + 1];
    acc.tz[p] = A.tgt[3 * ti + 2];
#pragma unroll
    for (int q = 0; q < kRun; ++q) acc.a[p][q][0] = acc.a[p][q][1] = acc.a[p][q][2] = 0.0;
  }
  const int64_t L = A.range_total;
  const int64_t lo = L * blockIdx.y / A.n_splits, hi = L * (blockIdx.y + 1) / A.n_splits;
  int64_t pos = 0;
  for (int r = 0; r < A.n_ranges && pos < hi; ++r) {
    const SrcRange R = A.ranges[r];
    const int64_t len = R.end - R.begin;
    const int64_t a = max<int64_t>(lo - pos, 0), b = min<int64_t>(hi - pos, len);
    pos += len;
    if (a >= b) continue;
    const int64_t j0 = R.begin + a, j1 = R.begin + b;
    const int64_t s0 = A.meta[k].k0[R.block], s1 = s0 + A.meta[k].kn[R.block];
    run_block_b<kTpl, kRun>(R.block, A, q0, j0, min(j1, s0), acc);
    run_block_b<kTpl, kRun>(R.block, A, q0, max(j0, s1), j1, acc);
  }
#pragma unroll
  for (int p = 0; p < kTpl; ++p) {
    const int i = lane + kWave * p;
    if (i < tc) {
#pragma unroll
      for (int q = 0; q < kRun; ++q) {
        if (q0 + q >= A.nrhs) break;
        double *out = A.part + ((int64_t)blockIdx.y * A.nrhs + q0 + q) * A.T * 3;
        const int64_t o = 3 * ((int64_t)t0 + i);
        out[o] = 0.5 * acc.a[p][q][0];   // the pairs add twice the velocity
        out[o + 1] = 0.5 * acc.a[p][q][1];
        out[o + 2] = 0.5 * acc.a[p][q][2];
      }
    }
  }
}

// Equivalent-source far field, many right-hand sides (SMFS_MIXED_EQ).
// q32b[((q n_eq + j) nrhs + v) 3 + c] = (float) (E lambda_hat_v(free sphere q))[3 j + c]:
// one thread per row of E, one contact-free sphere and kRun vectors
// (blockIdx.y, blockIdx.z); the strengths are wave-uniform.
template <int kRun>
__global__ __launch_bounds__(256) void k_eq_strengths_block(const double *__restrict__ E, int32_t rows,
                                                            int32_t cols, const double *__restrict__ lamb,
                                                            int32_t nrhs, const SphereMeta *__restrict__ meta,
                                                            const int32_t *__restrict__ free_ids,
                                                            float *__restrict__ q32b) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y, v0 = blockIdx.z * kRun;
  const int ks = uniform(free_ids[q]);
  const ConstPtr l = (ConstPtr)(lamb + (int64_t)meta[ks].k0[0] * nrhs * 3);
  const int rr = r < rows ? r : 0;
  double acc[kRun];
#pragma unroll
  for (int v = 0; v < kRun; ++v) acc[v] = 0.0;
  for (int i = 0; i < cols; ++i) {
    const double e = E[(int64_t)i * rows + rr];
    const int j = i / 3, c = i - 3 * (i / 3);
#pragma unroll
    for (int v = 0; v < kRun; ++v) {
      const int vv = min(v0 + v, nrhs - 1);
      acc[v] = fma(e, l[((int64_t)j * nrhs + vv) * 3 + c], acc[v]);
    }
  }
  if (r >= rows) return;
  const int j = r / 3, c = r - 3 * (r / 3);
  const int ne = rows / 3;
#pragma unroll
  for (int v = 0; v < kRun; ++v)
    if (v0 + v < nrhs) q32b[(((int64_t)q * ne + j) * nrhs + v0 + v) * 3 + c] = (float)acc[v];
}

// The n_eq equivalent sources of one contact-free sphere for a run of kRun
// vectors at the slots' targets ux (relative to its centre; kOffSlot for a
// slot it must not reach); str points at the sphere's strengths
// [j][nrhs][3], q0 the run's first vector.
template <int kTpl, int kRun>
__device__ __forceinline__ void eq_sphere_block(ConstPtr32 pts, ConstPtr32 str, int ne, int nrhs, int q0,
                                                const float (&ux)[kTpl], const float (&uy)[kTpl],
                                                const float (&uz)[kTpl], float (&a)[kTpl][kRun][3]) {
  for (int j = 0; j < ne; ++j) {
    const ConstPtr32 ps = pts + 3 * j, pf = str + ((int64_t)j * nrhs + q0) * 3;
    const float sx = ps[0], sy = ps[1], sz = ps[2];
    float f[kRun][3];
#pragma unroll
    for (int q = 0; q < kRun; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) f[q][c] = pf[3 * q + c];
#pragma unroll
    for (int p = 0; p < kTpl; ++p) {
      const float rx = ux[p] - sx, ry = uy[p] - sy, rz = uz[p] - sz;
      const float r2 = fmaf(rx, rx, fmaf(ry, ry, rz * rz));
      const float ri = __builtin_amdgcn_rsqf(r2);
      const float ri2 = ri * ri;
#pragma unroll
      for (int q = 0; q < kRun; ++q) {
        const float t = fmaf(rx, f[q][0], fmaf(ry, f[q][1], rz * f[q][2])) * ri2;
        a[p][q][0] = fmaf(fmaf(rx, t, f[q][0]), ri, a[p][q][0]);
        a[p][q][1] = fmaf(fmaf(ry, t, f[q][1]), ri, a[p][q][1]);
        a[p][q][2] = fmaf(fmaf(rz, t, f[q][2]), ri, a[p][q][2]);
      }
    }
  }
}

// The FP32 equivalent-source sum for a run of kRun vectors (blockIdx.z) on
// the packed target tiles, the contact-free spheres split over blockIdx.y:
// each slot skips its own sphere and its sphere's near list, and the
// coordinates are formed, as in far_eq_wave.
template <int kTpl, int kRun>
__global__ __launch_bounds__(kBlock) void k_far_eq_block_f32(EqArgs A, const float *__restrict__ q32b,
                                                             int32_t nrhs, float *__restrict__ part32b) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t tile = (int64_t)blockIdx.x * kWavesPerBlock + uniform(threadIdx.x / kWave);
  if (tile >= A.n_tiles) return;
  const int4 tl = A.tiles[tile];
  const int t0 = uniform(tl.y), tc = uniform(tl.z);
  if (tc <= 0) return;
  const int q0 = blockIdx.z * kRun;
  const int split = blockIdx.y;
  const int f0 = uniform((int)((int64_t)A.n_free * split / A.n_splits));
  const int f1 = uniform((int)((int64_t)A.n_free * (split + 1) / A.n_splits));
  double tx[kTpl], ty[kTpl], tz[kTpl];  // targets, absolute
  float a[kTpl][kRun][3];
  int own[kTpl], e[kTpl], next[kTpl];
#pragma unroll
  for (int p = 0; p < kTpl; ++p) {
    const int i = lane + kWave * p;
    const int64_t ti = (int64_t)t0 + (i < tc ? i : 0);
    tx[p] = A.tgt[3 * ti];
    ty[p] = A.tgt[3 * ti + 1];
    tz[p] = A.tgt[3 * ti + 2];
#pragma unroll
    for (int q = 0; q < kRun; ++q) a[p][q][0] = a[p][q][1] = a[p][q][2] = 0.f;
    const int k = A.tsph[ti];
    own[p] = k;
    e[p] = A.near_off[k];
    const int e1 = A.near_off[k + 1];
    while (e[p] < e1 && A.near_idx[e[p]] < f0) ++e[p];
    next[p] = e[p] < e1 ? A.near_idx[e[p]] : 0x7fffffff;
  }
  const ConstPtr32 pts = (ConstPtr32)A.eqpt32;
  const int ne = A.n_eq;
  for (int fq = f0; fq < f1; ++fq) {
    const int ks = uniform(A.free_ids[fq]);
    bool on[kTpl];
    bool any_on = false;
#pragma unroll
    for (int p = 0; p < kTpl; ++p) {
      const bool near = fq == next[p];
      if (near) {
        ++e[p];
        next[p] = e[p] < A.near_off[own[p] + 1] ? A.near_idx[e[p]] : 0x7fffffff;
      }
      on[p] = !near && ks != own[p];
      any_on = any_on || on[p];
    }
    if (!__any(any_on)) continue;
    const double sx = A.centers[3 * ks], sy = A.centers[3 * ks + 1], sz = A.centers[3 * ks + 2];
    float ux[kTpl], uy[kTpl], uz[kTpl];
#pragma unroll
    for (int p = 0; p < kTpl; ++p) {
      ux[p] = on[p] ? (float)(tx[p] - sx) : kOffSlot;
      uy[p] = on[p] ? (float)(ty[p] - sy) : kOffSlot;
      uz[p] = on[p] ? (float)(tz[p] - sz) : kOffSlot;
    }
    const ConstPtr32 str = (ConstPtr32)(q32b + (int64_t)fq * ne * nrhs * 3);
    eq_sphere_block<kTpl, kRun>(pts, str, ne, nrhs, q0, ux, uy, uz, a);
  }
#pragma unroll
  for (int p = 0; p < kTpl; ++p) {
    const int i = lane + kWave * p;
    if (i < tc) {
#pragma unroll
      for (int q = 0; q < kRun; ++q) {
        if (q0 + q >= nrhs) break;
        float *out = part32b + ((int64_t)split * nrhs + q0 + q) * A.T * 3;
        const int64_t o = 3 * ((int64_t)t0 + i);
        out[o] = a[p][q][0];
        out[o + 1] = a[p][q][1];
        out[o + 2] = a[p][q][2];
      }
    }
  }
}

// FP64 sum of the near contact-free proxies (near lists) for a run of kRun
// vectors (blockIdx.z) into one partial slice out [nrhs][T][3].
template <int kTpl, int kRun>
__global__ __launch_bounds__(kBlock) void k_near_block_f64(BlockDirectArgs A, const int32_t *__restrict__ free_ids,
                                                           const int32_t *__restrict__ near_off,
                                                           const int32_t *__restrict__ near_idx,
                                                           double *__restrict__ out) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t tile = (int64_t)blockIdx.x * kWavesPerBlock + uniform(threadIdx.x / kWave);
  if (tile >= A.n_tiles) return;
  const int4 tl = A.tiles[tile];
  const int k = uniform(tl.x), t0 = uniform(tl.y), tc = uniform(tl.z);
  const int q0 = blockIdx.z * kRun;
  AccB<kTpl, kRun> acc;
#pragma unroll
  for (int p = 0; p < kTpl; ++p) {
    const int i = lane + kWave * p;
    const int64_t ti = (int64_t)t0 + (i < tc ? i : 0);
    acc.tx[p] = A.tgt[3 * ti];
    acc.ty[p] = A.tgt[3 * ti + 1];
    acc.tz[p] = A.tgt[3 * ti + 2];
#pragma unroll
    for (int q = 0; q < kRun; ++q) acc.a[p][q][0] = acc.a[p][q][1] = acc.a[p][q][2] = 0.0;
  }
  const int e0 = uniform(near_off[k]), e1 = uniform(near_off[k + 1]);
  for (int e = e0; e < e1; ++e) {
    const int ks = uniform(free_ids[uniform(near_idx[e])]);
    const int j0 = uniform((int)A.meta[ks].k0[0]);
    const int j1 = j0 + uniform(A.meta[ks].kn[0]);
    run_sources_block<kTpl, kRun, 0>(A.src, A.lamb, A.nrhs, q0, j0, j1, acc);
  }
#pragma unroll
  for (int p = 0; p < kTpl; ++p) {
    const int i = lane + kWave * p;
    if (i < tc) {
#pragma unroll
      for (int q = 0; q < kRun; ++q) {
        if (q0 + q >= A.nrhs) break;
        double *o3 = out + (int64_t)(q0 + q) * A.T * 3;
        const int64_t o = 3 * ((int64_t)t0 + i);
        o3[o] = 0.5 * acc.a[p][q][0];   // the pairs add twice the velocity
        o3[o + 1] = 0.5 * acc.a[p][q][1];
        o3[o + 2] = 0.5 * acc.a[p][q][2];
      }
    }
  }
}

// Mixed precision, many right-hand sides: the FP32 far field of the
// contact-free proxies for a run of kRun vectors (blockIdx.z), one-sphere
// tiles, the free spheres split over blockIdx.y.  Coordinates relative to
// sphere centres as in far_wave; every pair's separation and 1/|r| serve the
// whole run.  Strengths str32 are source-major, [proxy][nrhs][3].
template <int kTpl, int kRun>
__global__ __launch_bounds__(kBlock) void k_far_block_f32(Far32Args A, const float *__restrict__ str32b,
                                                          int32_t nrhs, float *__restrict__ part32b) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t tile = (int64_t)blockIdx.x * kWavesPerBlock + uniform(threadIdx.x / kWave);
  if (tile >= A.n_tiles) return;
  const int4 tl = A.tiles[tile];
  const int k = uniform(tl.x), t0 = uniform(tl.y), tc = uniform(tl.z);
  const int q0 = blockIdx.z * kRun;
  const int split = blockIdx.y;
  float tx[kTpl], ty[kTpl], tz[kTpl], a[kTpl][kRun][3];
#pragma unroll
  for (int p = 0; p < kTpl; ++p) {
    const int i = lane + kWave * p;
    const int64_t ti = (int64_t)t0 + (i < tc ? i : 0);
    tx[p] = A.tgt32[3 * ti];
    ty[p] = A.tgt32[3 * ti + 1];
    tz[p] = A.tgt32[3 * ti + 2];
#pragma unroll
    for (int q = 0; q < kRun; ++q) a[p][q][0] = a[p][q][1] = a[p][q][2] = 0.f;
  }
  const ConstPtr32 src = (ConstPtr32)A.src32, str = (ConstPtr32)str32b;
  const double ckx = A.centers[3 * k], cky = A.centers[3 * k + 1], ckz = A.centers[3 * k + 2];
  const int f0 = uniform((int)((int64_t)A.n_free * split / A.n_splits));
  const int f1 = uniform((int)((int64_t)A.n_free * (split + 1) / A.n_splits));
  const int np = A.n_proxy;
  for (int fq = f0; fq < f1; ++fq) {
    const int ks = A.free_ids[fq];
    if (ks == k) continue;
    const float dx = (float)(A.centers[3 * ks] - ckx), dy = (float)(A.centers[3 * ks + 1] - cky),
                dz = (float)(A.centers[3 * ks + 2] - ckz);
    float ux[kTpl], uy[kTpl], uz[kTpl];
#pragma unroll
    for (int p = 0; p < kTpl; ++p) {
      ux[p] = tx[p] - dx;
      uy[p] = ty[p] - dy;
      uz[p] = tz[p] - dz;
    }
    const int j1 = uniform(ks * np + np);
    for (int j = uniform(ks * np); j < j1; ++j) {
      const ConstPtr32 ps = src + 3 * j, pf = str + ((int64_t)j * nrhs + q0) * 3;
      const float sx = ps[0], sy = ps[1], sz = ps[2];
      float f[kRun][3];
#pragma unroll
      for (int q = 0; q < kRun; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) f[q][c] = pf[3 * q + c];
#pragma unroll
      for (int p = 0; p < kTpl; ++p) {
        const float rx = ux[p] - sx, ry = uy[p] - sy, rz = uz[p] - sz;
        const float r2 = fmaf(rx, rx, fmaf(ry, ry, rz * rz));
        const float ri = __builtin_amdgcn_rsqf(r2);
        const float ri2 = ri * ri;
#pragma unroll
        for (int q = 0; q < kRun; ++q) {
          const float t = fmaf(rx, f[q][0], fmaf(ry, f[q][1], rz * f[q][2])) * ri2;
          a[p][q][0] = fmaf(fmaf(rx, t, f[q][0]), ri, a[p][q][0]);
          a[p][q][1] = fmaf(fmaf(ry, t, f[q][1]), ri, a[p][q][1]);
          a[p][q][2] = fmaf(fmaf(rz, t, f[q][2]), ri, a[p][q][2]);
        }
      }
    }
  }
#pragma unroll
  for (int p = 0; p < kTpl; ++p) {
    const int i = lane + kWave * p;
    if (i < tc) {
#pragma unroll
      for (int q = 0; q < kRun; ++q) {
        if (q0 + q >= nrhs) break;
        float *out = part32b + ((int64_t)split * nrhs + q0 + q) * A.T * 3;
        const int64_t o = 3 * ((int64_t)t0 + i);
        out[o] = a[p][q][0];
        out[o + 1] = a[p][q][1];
        out[o + 2] = a[p][q][2];
      }
    }
  }
}

// y_q = mu_q + W c0 (sum_split part[split][q] + sum_split part32[split][q])
__global__ void k_reduce_block(int64_t n3, int32_t nrhs, int32_t ns, const double *__restrict__ part,
                               int32_t ns32, const float *__restrict__ part32,
                               const double *__restrict__ base, int64_t ldb,
                               const double *__restrict__ sw, double c0, double *__restrict__ y,
                               int64_t ldy) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (i >= n3 || q >= nrhs) return;
  double acc = 0.0;
  for (int s = 0; s < ns; ++s) acc += part[((int64_t)s * nrhs + q) * n3 + i];
  for (int s = 0; s < ns32; ++s) acc += (double)part32[((int64_t)s * nrhs + q) * n3 + i];
  y[q * ldy + i] = base[q * ldb + i] + sw[i / 3] * c0 * acc;
}

// Batched GMRES helpers: blockIdx.z selects the right-hand side; vector j of
// system q lives at V + (j * nrhs + q) * ld.
__global__ __launch_bounds__(kBlock) void k_mdot_b(const double *__restrict__ V, int64_t ld,
                                                   int32_t nrhs, int32_t nv,
                                                   const double *__restrict__ W, int64_t ldw,
                                                   int64_t n, int64_t chunk,
                                                   double *__restrict__ part, int32_t nchunks) {
  __shared__ double sh[kDotVecs][kWavesPerBlock];
  const int c = blockIdx.x, q = blockIdx.z;
  const int j0 = blockIdx.y * kDotVecs;
  const double *w = W + q * ldw;
  const int64_t b = (int64_t)c * chunk, e = min(n, b + chunk);
  double acc[kDotVecs];
#pragma unroll
  for (int s = 0; s < kDotVecs; ++s) acc[s] = 0.0;
  for (int64_t i = b + threadIdx.x; i < e; i += kBlock) {
    const double wi = w[i];
#pragma unroll
    for (int s = 0; s < kDotVecs; ++s)
      if (j0 + s < nv) acc[s] = fma(V[((int64_t)(j0 + s) * nrhs + q) * ld + i], wi, acc[s]);
  }
  block_sum<kDotVecs>(acc, sh);
  if (threadIdx.x < kDotVecs && j0 + (int)threadIdx.x < nv)
    part[((int64_t)q * nv + j0 + threadIdx.x) * nchunks + c] = acc[threadIdx.x];
}

__global__ void k_mdot_final_b(int32_t nrhs, int32_t nv, const double *__restrict__ part,
                               int32_t nchunks, double *__restrict__ h, int32_t ldh) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x, q = blockIdx.y;
  if (j >= nv) return;
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += part[((int64_t)q * nv + j) * nchunks + c];
  h[(int64_t)q * ldh + j] = s;
}

__global__ void k_mupdate_b(const double *__restrict__ V, int64_t ld, int32_t nrhs, int32_t nv,
                            const double *__restrict__ h, int32_t ldh, double *__restrict__ W,
                            int64_t ldw, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (i >= n) return;
  W[q * ldw + i] -= basis_row_dot(V + (int64_t)q * ld, (int64_t)nrhs * ld, nv, h + (int64_t)q * ldh, i);
}

__global__ __launch_bounds__(kBlock) void k_sumsq_b(const double *__restrict__ W, int64_t ldw,
                                                    int64_t n, int64_t chunk,
                                                    double *__restrict__ part, int32_t nchunks) {
  __shared__ double sh[1][kWavesPerBlock];
  const int q = blockIdx.y;
  const double *w = W + q * ldw;
  const int64_t b = (int64_t)blockIdx.x * chunk, e = min(n, b + chunk);
  double acc[1] = {0.0};
  for (int64_t i = b + threadIdx.x; i < e; i += kBlock) acc[0] = fma(w[i], w[i], acc[0]);
  block_sum<1>(acc, sh);
  if (threadIdx.x == 0) part[(int64_t)q * nchunks + blockIdx.x] = acc[0];
}

// beta[q * ldb] = sqrt(sum of parts); then w_q /= beta_q (0 when beta = 0)
__global__ void k_sqrt_final_b(int32_t nrhs, const double *__restrict__ part, int32_t nchunks,
                               double *__restrict__ beta, int32_t ldb) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nrhs) return;
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += part[(int64_t)q * nchunks + c];
  beta[(int64_t)q * ldb] = sqrt(s);
}

__global__ void k_scale_b(double *__restrict__ W, int64_t ldw, int64_t n,
                          const double *__restrict__ beta, int32_t ldb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (i >= n) return;
  const double b = beta[(int64_t)q * ldb];
  W[q * ldw + i] = b > 0.0 ? W[q * ldw + i] / b : 0.0;
}

// x_q += sum_j V[j][q] c[q][j]
__global__ void k_combine_b(const double *__restrict__ V, int64_t ld, int32_t nrhs, int32_t nv,
                            const double *__restrict__ cf, int32_t ldc, double *__restrict__ X,
                            int64_t ldx, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (i >= n) return;
  X[q * ldx + i] += basis_row_dot(V + (int64_t)q * ld, (int64_t)nrhs * ld, nv, cf + (int64_t)q * ldc, i);
}

}  // namespace

hipError_t launch_pinv_block(const int4 *utasks, int64_t nu, const int4 *vtasks, int64_t nv,
                             const SphereMeta *meta, const FactorSlot *fs, const double *fac,
                             const double *mu, int64_t ldmu, int32_t nrhs, double *S, int64_t lds,
                             double *lamb, double dscale, hipStream_t s) {
  // one workgroup per 64-row task and 64 right-hand sides
  const unsigned qt = (unsigned)((nrhs + kGT - 1) / kGT);
  if (nu > 0)
    hipLaunchKernelGGL(k_pinv_block_u, dim3((unsigned)nu, qt), dim3(kBlock), 0, s, utasks, nu, meta, fs, fac, mu,
                       ldmu, nrhs, S, lds);
  if (nv > 0)
    hipLaunchKernelGGL(k_pinv_block_v, dim3((unsigned)nv, qt), dim3(kBlock), 0, s, vtasks, nv, meta, fs, fac, S,
                       lds, nrhs, lamb, dscale);
  return hipGetLastError();
}

hipError_t launch_eq_block(const BlockDirectArgs &d, const EqArgs &f, const double *E, int32_t n_proxy,
                           float *q32b, double *near_out, float *part32b, hipStream_t s) {
  if (f.n_free <= 0 || d.nrhs == 0) return hipSuccess;
  const unsigned nz = (unsigned)((d.nrhs + kBlockRun - 1) / kBlockRun);
  const int rows = 3 * f.n_eq;
  hipLaunchKernelGGL((k_eq_strengths_block<kBlockRun>), dim3((unsigned)((rows + 255) / 256), (unsigned)f.n_free, nz),
                     dim3(256), 0, s, E, rows, 3 * n_proxy, d.lamb, d.nrhs, d.meta, f.free_ids, q32b);
  if (d.n_tiles > 0) {
    const unsigned nb = (unsigned)((d.n_tiles + kWavesPerBlock - 1) / kWavesPerBlock);
    hipLaunchKernelGGL((k_near_block_f64<kDirectTpl, kBlockRun>), dim3(nb, 1, nz), dim3(kBlock), 0, s, d,
                       f.free_ids, f.near_off, f.near_idx, near_out);
    if (f.n_splits > 0 && f.n_tiles > 0)
      hipLaunchKernelGGL((k_far_eq_block_f32<kDirectTpl, kBlockRun>),
                         dim3((unsigned)((f.n_tiles + kWavesPerBlock - 1) / kWavesPerBlock), (unsigned)f.n_splits, nz),
                         dim3(kBlock), 0, s, f, q32b, d.nrhs, part32b);
  }
  return hipGetLastError();
}

hipError_t launch_direct_block(const BlockDirectArgs &a, hipStream_t s) {
  if (a.n_tiles == 0 || a.nrhs == 0) return hipSuccess;
  dim3 grid((unsigned)((a.n_tiles + kWavesPerBlock - 1) / kWavesPerBlock), (unsigned)a.n_splits,
            (unsigned)((a.nrhs + kBlockRun - 1) / kBlockRun));
  hipLaunchKernelGGL((k_direct_block<kDirectTpl, kBlockRun>), grid, dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_reduce_block(int64_t n3, int32_t nrhs, int32_t ns, const double *part, int32_t ns32,
                               const float *part32, const double *base, int64_t ldb, const double *sw,
                               double c0, double *y, int64_t ldy, hipStream_t s) {
  if (n3 == 0 || nrhs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_block, dim3(blocks_for(n3), nrhs), dim3(kBlock), 0, s, n3, nrhs, ns,
                     part, ns32, part32, base, ldb, sw, c0, y, ldy);
  return hipGetLastError();
}

hipError_t launch_far_block_f32(const Far32Args &a, const float *str32b, int32_t nrhs, float *part32b,
                                hipStream_t s) {
  if (a.n_tiles == 0 || a.n_splits == 0 || nrhs == 0) return hipSuccess;
  dim3 grid((unsigned)((a.n_tiles + kWavesPerBlock - 1) / kWavesPerBlock), (unsigned)a.n_splits,
            (unsigned)((nrhs + kBlockRun - 1) / kBlockRun));
  hipLaunchKernelGGL((k_far_block_f32<kDirectTpl, kBlockRun>), grid, dim3(kBlock), 0, s, a, str32b, nrhs,
                     part32b);
  return hipGetLastError();
}

hipError_t launch_arnoldi_block(const double *V, int64_t ld, int32_t nrhs, int32_t nv, double *W,
                                int64_t n, double *part, int32_t nchunks, double *h, int32_t ldh,
                                hipStream_t s) {
  // h_q = V_q^T w_q ; w_q -= V_q h_q
  const int64_t chunk = chunk_len(n, nchunks);
  dim3 g1((unsigned)nchunks, (unsigned)((nv + kDotVecs - 1) / kDotVecs), (unsigned)nrhs);
  hipLaunchKernelGGL(k_mdot_b, g1, dim3(kBlock), 0, s, V, ld, nrhs, nv, W, ld, n, chunk, part, nchunks);
  hipLaunchKernelGGL(k_mdot_final_b, dim3(blocks_for(nv), nrhs), dim3(kBlock), 0, s, nrhs, nv, part,
                     nchunks, h, ldh);
  hipLaunchKernelGGL(k_mupdate_b, dim3(blocks_for(n), nrhs), dim3(kBlock), 0, s, V, ld, nrhs, nv, h,
                     ldh, W, ld, n);
  return hipGetLastError();
}

hipError_t launch_norm_scale_block(double *W, int64_t ld, int32_t nrhs, int64_t n, double *part,
                                   int32_t nchunks, double *beta, int32_t ldb, bool scale,
                                   hipStream_t s) {
  const int64_t chunk = chunk_len(n, nchunks);
  hipLaunchKernelGGL(k_sumsq_b, dim3(nchunks, nrhs), dim3(kBlock), 0, s, W, ld, n, chunk, part, nchunks);
  hipLaunchKernelGGL(k_sqrt_final_b, dim3(blocks_for(nrhs)), dim3(kBlock), 0, s, nrhs, part, nchunks,
                     beta, ldb);
  if (scale)
    hipLaunchKernelGGL(k_scale_b, dim3(blocks_for(n), nrhs), dim3(kBlock), 0, s, W, ld, n, beta, ldb);
  return hipGetLastError();
}

hipError_t launch_scale_block(double *W, int64_t ld, int32_t nrhs, int64_t n, const double *beta,
                              int32_t ldb, hipStream_t s) {
  if (n == 0 || nrhs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_b, dim3(blocks_for(n), nrhs), dim3(kBlock), 0, s, W, ld, n, beta, ldb);
  return hipGetLastError();
}

hipError_t launch_combine_block(const double *V, int64_t ld, int32_t nrhs, int32_t nv,
                                const double *cf, int32_t ldc, double *X, int64_t ldx, int64_t n,
                                hipStream_t s) {
  if (nv <= 0 || n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_combine_b, dim3(blocks_for(n), nrhs), dim3(kBlock), 0, s, V, ld, nrhs, nv, cf,
                     ldc, X, ldx, n);
  return hipGetLastError();
}

}  // namespace smfs

// ===========================================================================
// Serving: one launch covers the products (and the Arnoldi steps) of many
// independent problems, each described by a ServeDesc.  Flat work indices
// (tiles, pseudo-inverse rows) are mapped to their problem by a binary
// search over the per-problem prefixes; per-problem element loops use the
// problem index as a grid dimension.

namespace smfs {
namespace {

// Largest r with key(r) <= t (prefixes are non-decreasing, key(0) = 0).
template <typename Key>
__device__ __forceinline__ int find_problem(int32_t nprob, int64_t t, Key key) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (key(mid) <= t) lo = mid;
    else hi = mid - 1;
  }
  return uniform(lo);
}

// A request takes part in a launch while its cycle state is active; the
// product reads V[j] and writes V[j + 1] of its basis.
__device__ __forceinline__ bool serve_on(const ServeDesc &d) { return uniform(d.gv->active) != 0; }
__device__ __forceinline__ int serve_j(const ServeDesc &d) { return uniform(d.gv->j); }

__global__ __launch_bounds__(kBlock) void k_serve_pinv_u(const ServeDesc *__restrict__ D,
                                                         int32_t nprob, int64_t total) {
  const int64_t t = (int64_t)blockIdx.x * kWavesPerBlock + uniform(threadIdx.x / kWave);
  if (t >= total) return;
  const int r = find_problem(nprob, t, [D](int i) { return D[i].utask0; });
  const ServeDesc &d = D[r];
  const int64_t tl = t - d.utask0;
  if (tl >= d.n_utask || !serve_on(d)) return;
  const double *x = d.V + (int64_t)serve_j(d) * d.ld;
  pinv_u_row(d.utask, tl, d.da.meta, d.fs, d.fac, x, d.sbuf);
}

__global__ __launch_bounds__(kBlock) void k_serve_pinv_v(const ServeDesc *__restrict__ D,
                                                         int32_t nprob, int64_t total) {
  const int64_t t = (int64_t)blockIdx.x * kWavesPerBlock + uniform(threadIdx.x / kWave);
  if (t >= total) return;
  const int r = find_problem(nprob, t, [D](int i) { return D[i].vtask0; });
  const ServeDesc &d = D[r];
  const int64_t tl = t - d.vtask0;
  if (tl >= d.n_vtask || !serve_on(d)) return;
  pinv_v_row(d.vtask, tl, d.da.meta, d.fs, d.fac, d.sbuf, d.lam, d.da.dscale);
}

template <int kTpl>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(SMFS_DIRECT_WAVES, 8))) void k_serve_direct(const ServeDesc *__restrict__ D, int32_t nprob,
                                                                  int64_t total) {
  const int64_t t = (int64_t)blockIdx.x * kWavesPerBlock + uniform(threadIdx.x / kWave);
  if (t >= total) return;
  const int r = find_problem(nprob, t, [D](int i) { return D[i].tile0; });
  const ServeDesc &d = D[r];
  if ((int)blockIdx.y >= d.da.n_splits || !serve_on(d)) return;
  direct_wave<kTpl, false>(d.da, t - d.tile0, blockIdx.y);
}

// Mixed precision: FP32 copies of the proxy strengths of every problem.
__global__ void k_serve_to32(const ServeDesc *__restrict__ D) {
  const ServeDesc &d = D[blockIdx.y];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d.fa.n_splits == 0 || i >= d.n_str32 || !serve_on(d)) return;
  d.str32[i] = (float)d.lam[i];
}

// Mixed precision: FP32 far field of the contact-free proxies, every
// problem's one-sphere tiles in one launch (flat index over the problems'
// tiles, split in blockIdx.y).
template <int kTpl>
__global__ __launch_bounds__(kBlock) void k_serve_far32(const ServeDesc *__restrict__ D, int32_t nprob,
                                                        int64_t total) {
  const int64_t t = (int64_t)blockIdx.x * kWavesPerBlock + uniform(threadIdx.x / kWave);
  if (t >= total) return;
  const int r = find_problem(nprob, t, [D](int i) { return D[i].stile0; });
  const ServeDesc &d = D[r];
  if ((int)blockIdx.y >= d.fa.n_splits || !serve_on(d)) return;
  far_wave<kTpl>(d.fa, t - d.stile0, blockIdx.y);
}

// V[j + 1] = x + W c0 (sum_s part[s] + sum_s part32[s]) with x = V[j] (the
// same arithmetic as k_reduce_epilogue)
__global__ void k_serve_reduce(const ServeDesc *__restrict__ D) {
  const ServeDesc &d = D[blockIdx.y];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n || !serve_on(d)) return;
  const int64_t j = serve_j(d);
  const int32_t ns = d.da.n_splits;
  double acc = 0.0;
  for (int s = 0; s < ns; ++s) acc += d.da.part[(int64_t)s * d.n + i];
  for (int s = 0; s < d.fa.n_splits; ++s) acc += (double)d.fa.part32[(int64_t)s * d.n + i];
  double v = d.c0 * acc;
  v *= d.sw[i / 3];
  v += d.V[j * d.ld + i];
  d.V[(j + 1) * d.ld + i] = v;
}

// Classical Gram-Schmidt pass of w = V[j + 1] against V[0..j] of every
// problem (pass 0 writes h, pass 1 writes h2), with the chunking and
// summation order of the single-problem kernels.
__global__ __launch_bounds__(kBlock) void k_serve_mdot(const ServeDesc *__restrict__ D) {
  __shared__ double sh[kDotVecs][kWavesPerBlock];
  const ServeDesc &d = D[blockIdx.z];
  if (!serve_on(d)) return;   // uniform over the block
  const int c = blockIdx.x;
  const int j0 = blockIdx.y * kDotVecs;
  const int nv = serve_j(d) + 1;
  if (c >= d.nch || j0 >= nv) return;   // uniform over the block
  const int64_t chunk = chunk_len(d.n, d.nch);
  const int64_t b = (int64_t)c * chunk, e = min(d.n, b + chunk);
  const double *w = d.V + (int64_t)nv * d.ld;
  double acc[kDotVecs];
#pragma unroll
  for (int q = 0; q < kDotVecs; ++q) acc[q] = 0.0;
  for (int64_t i = b + threadIdx.x; i < e; i += kBlock) {
    const double wi = w[i];
#pragma unroll
    for (int q = 0; q < kDotVecs; ++q)
      if (j0 + q < nv) acc[q] = fma(d.V[(int64_t)(j0 + q) * d.ld + i], wi, acc[q]);
  }
  block_sum<kDotVecs>(acc, sh);
  if (threadIdx.x < kDotVecs && j0 + (int)threadIdx.x < nv)
    d.red[(int64_t)(j0 + threadIdx.x) * d.nch + c] = acc[threadIdx.x];
}

__global__ void k_serve_mdot_final(const ServeDesc *__restrict__ D, int pass) {
  const ServeDesc &d = D[blockIdx.y];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (!serve_on(d) || j >= serve_j(d) + 1) return;
  double s = 0.0;
  for (int c = 0; c < d.nch; ++c) s += d.red[(int64_t)j * d.nch + c];
  (pass ? d.h2 : d.h)[j] = s;
}

__global__ void k_serve_mupdate(const ServeDesc *__restrict__ D, int pass) {
  const ServeDesc &d = D[blockIdx.y];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n || !serve_on(d)) return;
  const int nv = serve_j(d) + 1;
  d.V[(int64_t)nv * d.ld + i] -= basis_row_dot(d.V, d.ld, nv, pass ? d.h2 : d.h, i);
}

__global__ __launch_bounds__(kBlock) void k_serve_sumsq(const ServeDesc *__restrict__ D) {
  __shared__ double sh[1][kWavesPerBlock];
  const ServeDesc &d = D[blockIdx.y];
  if ((int)blockIdx.x >= d.nch || !serve_on(d)) return;
  const int64_t chunk = chunk_len(d.n, d.nch);
  const int64_t b = (int64_t)blockIdx.x * chunk, e = min(d.n, b + chunk);
  const double *y = d.V + (int64_t)(serve_j(d) + 1) * d.ld;
  double acc[1] = {0.0};
  for (int64_t i = b + threadIdx.x; i < e; i += kBlock) acc[0] = fma(y[i], y[i], acc[0]);
  block_sum<1>(acc, sh);
  if (threadIdx.x == 0) d.red[blockIdx.x] = acc[0];
}

__global__ void k_serve_norm(const ServeDesc *__restrict__ D, int32_t nprob) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nprob) return;
  const ServeDesc &d = D[r];
  if (!d.gv->active) return;
  double s = 0.0;
  for (int c = 0; c < d.nch; ++c) s += d.red[c];
  d.h[d.gv->j + 1] = sqrt(s);
}

__global__ void k_serve_scale(const ServeDesc *__restrict__ D) {
  const ServeDesc &d = D[blockIdx.y];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n || !serve_on(d)) return;
  const int nv = serve_j(d) + 1;
  const double b = d.h[nv];
  double *y = d.V + (int64_t)nv * d.ld;
  y[i] = b > 0.0 ? y[i] / b : 0.0;
}

// Givens step of one request per thread (the host form of the single-problem
// solver, on the device): the new column of H is h + h2 (the two
// Gram-Schmidt passes) with the norm below them; the earlier rotations are
// applied to it, a new rotation zeroes its last entry and rotates g.  The
// request stays active until the estimate |g[j+1]| / |b| meets the
// tolerance, the iteration limit is reached, the new vector vanishes
// (breakdown) or the cycle is full.
__global__ void k_serve_givens(const ServeDesc *__restrict__ D, int32_t nprob) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nprob) return;
  const ServeDesc &d = D[r];
  ServeGivens &q = *d.gv;
  if (!q.active) return;
  const int j = q.j, m = q.m;
  double *col = q.H + (int64_t)j * (m + 1);
  for (int k = 0; k <= j + 1; ++k) col[k] = d.h[k] + (k <= j ? d.h2[k] : 0.0);
  for (int k = 0; k < j; ++k) {
    const double t = q.cs[k] * col[k] + q.sn[k] * col[k + 1];
    col[k + 1] = -q.sn[k] * col[k] + q.cs[k] * col[k + 1];
    col[k] = t;
  }
  const double den = hypot(col[j], col[j + 1]);
  q.cs[j] = den > 0 ? col[j] / den : 1.0;
  q.sn[j] = den > 0 ? col[j + 1] / den : 0.0;
  col[j] = den;
  col[j + 1] = 0.0;
  q.g[j + 1] = -q.sn[j] * q.g[j];
  q.g[j] = q.cs[j] * q.g[j];
  q.j = j + 1;
  q.total += 1;
  q.est = fabs(q.g[j + 1]) / q.bnorm;
  q.breakdown = d.h[j + 1] == 0.0 ? 1 : 0;
  if (q.est <= q.tol || q.total >= q.max_it || q.breakdown || q.j == m) q.active = 0;
}

}  // namespace

hipError_t launch_serve_product(const ServeDesc *d, int32_t nprob, int64_t tiles, int64_t utasks,
                                int64_t vtasks, int32_t max_splits, int64_t max_n, int64_t stiles,
                                int32_t max_splits32, int64_t max_str32, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  if (utasks > 0)
    hipLaunchKernelGGL(k_serve_pinv_u, dim3(blocks_for(utasks, kWavesPerBlock)), dim3(kBlock), 0, s,
                       d, nprob, utasks);
  if (vtasks > 0)
    hipLaunchKernelGGL(k_serve_pinv_v, dim3(blocks_for(vtasks, kWavesPerBlock)), dim3(kBlock), 0, s,
                       d, nprob, vtasks);
  if (tiles > 0)
    hipLaunchKernelGGL((k_serve_direct<kDirectTpl>),
                       dim3(blocks_for(tiles, kWavesPerBlock), (unsigned)max_splits), dim3(kBlock), 0,
                       s, d, nprob, tiles);
  if (stiles > 0 && max_splits32 > 0) {
    hipLaunchKernelGGL(k_serve_to32, dim3(blocks_for(max_str32), nprob), dim3(kBlock), 0, s, d);
    hipLaunchKernelGGL((k_serve_far32<kDirectTpl>),
                       dim3(blocks_for(stiles, kWavesPerBlock), (unsigned)max_splits32), dim3(kBlock), 0,
                       s, d, nprob, stiles);
  }
  hipLaunchKernelGGL(k_serve_reduce, dim3(blocks_for(max_n), nprob), dim3(kBlock), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_serve_arnoldi(const ServeDesc *d, int32_t nprob, int32_t max_nv, int32_t max_nch,
                                int64_t max_n, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  const dim3 gd((unsigned)max_nch, (unsigned)((max_nv + kDotVecs - 1) / kDotVecs), (unsigned)nprob);
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(k_serve_mdot, gd, dim3(kBlock), 0, s, d);
    hipLaunchKernelGGL(k_serve_mdot_final, dim3(blocks_for(max_nv), nprob), dim3(kBlock), 0, s, d, pass);
    hipLaunchKernelGGL(k_serve_mupdate, dim3(blocks_for(max_n), nprob), dim3(kBlock), 0, s, d, pass);
  }
  hipLaunchKernelGGL(k_serve_sumsq, dim3((unsigned)max_nch, nprob), dim3(kBlock), 0, s, d);
  hipLaunchKernelGGL(k_serve_norm, dim3(blocks_for(nprob)), dim3(kBlock), 0, s, d, nprob);
  hipLaunchKernelGGL(k_serve_scale, dim3(blocks_for(max_n), nprob), dim3(kBlock), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_serve_givens(const ServeDesc *d, int32_t nprob, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_serve_givens, dim3(blocks_for(nprob)), dim3(kBlock), 0, s, d, nprob);
  return hipGetLastError();
}

}  // namespace smfs

// ===========================================================================
// The shared factor of the contact-free spheres (eq. transform with one
// B^+ for all of them) as two GEMMs on FP64 MFMA, the spheres as columns:
// S_q = Sigma^-1 U_0^T mu_q, then lambda_q = V_0 S_q.  One wave per 32 x 32
// tile (rows of U_0^T or V_0 by free spheres); the factor is read once per
// 32 spheres instead of once per sphere.

namespace smfs {
namespace {

__global__ __launch_bounds__(kBlock) void k_pinv_shared_u(const int32_t *__restrict__ free_ids,
                                                          int32_t n_free,
                                                          const SphereMeta *__restrict__ meta,
                                                          const FactorSlot *__restrict__ fs,
                                                          const double *__restrict__ fac,
                                                          const double *__restrict__ mu,
                                                          double *__restrict__ sbuf) {
  const int lane = threadIdx.x & 63;
  const FactorSlot &f = fs[0];
  const int rank = f.rank;
  const int r0 = ((int)blockIdx.x * kWavesPerBlock + uniform(threadIdx.x / kWave)) * 32;
  const int q0 = blockIdx.y * 32;
  if (r0 >= rank) return;
  const double *arow[2], *bcol[2];
  bool aok[2], bok[2];
  for (int h = 0; h < 2; ++h) {
    const int r = r0 + 16 * h + (lane & 15), q = q0 + 16 * h + (lane & 15);
    aok[h] = r < rank;
    bok[h] = q < n_free;
    arow[h] = fac + f.u_off + (int64_t)(aok[h] ? r : 0) * f.rows;
    bcol[h] = mu + 3 * meta[free_ids[bok[h] ? q : 0]].t0;
  }
  TileTN tile;
  mfma_tile_tn(arow, aok, bcol, bok, f.rows, tile);
  const double *sig = fac + f.sig_off;
  for (int ia = 0; ia < 2; ++ia)
    for (int jb = 0; jb < 2; ++jb)
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + 16 * ia + 4 * v + (lane >> 4), q = q0 + 16 * jb + (lane & 15);
        if (r < rank && q < n_free) sbuf[meta[free_ids[q]].s0 + r] = tile.acc[ia][jb][v] / sig[r];
      }
}

__global__ __launch_bounds__(kBlock) void k_pinv_shared_v(const int32_t *__restrict__ free_ids,
                                                          int32_t n_free,
                                                          const SphereMeta *__restrict__ meta,
                                                          const FactorSlot *__restrict__ fs,
                                                          const double *__restrict__ fac,
                                                          const double *__restrict__ sbuf,
                                                          double *__restrict__ lam, double dscale) {
  const int lane = threadIdx.x & 63;
  const FactorSlot &f = fs[0];
  const int rows = f.cols;
  const int r0 = ((int)blockIdx.x * kWavesPerBlock + uniform(threadIdx.x / kWave)) * 32;
  const int q0 = blockIdx.y * 32;
  if (r0 >= rows) return;
  const double *arow[2], *bcol[2];
  bool aok[2], bok[2];
  for (int h = 0; h < 2; ++h) {
    const int r = r0 + 16 * h + (lane & 15), q = q0 + 16 * h + (lane & 15);
    aok[h] = r < rows;
    bok[h] = q < n_free;
    arow[h] = fac + f.vt_off + (int64_t)(aok[h] ? r : 0) * f.cols;
    bcol[h] = sbuf + meta[free_ids[bok[h] ? q : 0]].s0;
  }
  TileTN tile;
  mfma_tile_tn(arow, aok, bcol, bok, f.rank, tile);
  for (int ia = 0; ia < 2; ++ia)
    for (int jb = 0; jb < 2; ++jb)
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + 16 * ia + 4 * v + (lane >> 4), q = q0 + 16 * jb + (lane & 15);
        if (r < rows && q < n_free) {
          const SphereMeta &m = meta[free_ids[q]];
          const int jl = r / 3, c = r - 3 * (r / 3);
          const double val = tile.acc[ia][jb][v];
          lam[3 * packed_index(m, jl) + c] = jl >= m.kn[0] + m.kn[1] + m.kn[2] ? val * dscale : val;
        }
      }
}

// The same two GEMMs in FP32 for the mixed form, on v_mfma_f32_16x16x4f32
// with FP32 accumulation.  Its operands take the layout of the FP64 form
// (lane l supplies A[i0 + l%16][k] and B[k][j0 + l%16] for k-slot l/16), but
// its result differs (measured on the device): register v of lane l holds
// C[i0 + 4 (l/16) + v][j0 + l%16].  B columns of another type are rounded
// to FP32 as they are loaded.  Successive 16-wide k chunks go to four
// accumulator sets in turn, added pairwise at the end: the shared factor's
// small singular values amplify rounding, and four shorter FP32 sums keep
// it near that of a strided dot product rather than one K/4-long chain.
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kAccSets = 4;

struct TileTN32 {
  f32x4 acc[2][2];
};

template <typename TB>
__device__ __forceinline__ void mfma_tile_tn32(const float *const arow[2], const bool aok[2],
                                               const TB *const bcol[2], const bool bok[2],
                                               int64_t K, TileTN32 &t) {
  const int lane = threadIdx.x & 63, g = lane >> 4;
  f32x4 acc[kAccSets][2][2];
#pragma unroll
  for (int u = 0; u < kAccSets; ++u)
#pragma unroll
    for (int ia = 0; ia < 2; ++ia)
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) acc[u][ia][jb] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int64_t kb = 0; kb < K; kb += 16 * kAccSets) {
#pragma unroll
    for (int u = 0; u < kAccSets; ++u) {
      const int64_t kc = kb + 16 * u;
      float a[2][4], b[2][4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int64_t k = kc + 4 * g + s;
        const bool kin = k < K;
#pragma unroll
        for (int ia = 0; ia < 2; ++ia) a[ia][s] = (aok[ia] && kin) ? arow[ia][k] : 0.f;
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) b[jb][s] = (bok[jb] && kin) ? (float)bcol[jb][k] : 0.f;
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int ia = 0; ia < 2; ++ia)
#pragma unroll
          for (int jb = 0; jb < 2; ++jb)
            acc[u][ia][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ia][s], b[jb][s], acc[u][ia][jb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int ia = 0; ia < 2; ++ia)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
      t.acc[ia][jb] = (acc[0][ia][jb] + acc[1][ia][jb]) + (acc[2][ia][jb] + acc[3][ia][jb]);
}

// s32 at each free sphere's s0 = Sigma^-1 U_0^T mu (FP32 copy fac32 of
// factor 0, whose FP64 offsets start at off0).
__global__ __launch_bounds__(kBlock) void k_pinv_shared_u32(const int32_t *__restrict__ free_ids,
                                                            int32_t n_free,
                                                            const SphereMeta *__restrict__ meta,
                                                            const FactorSlot *__restrict__ fs,
                                                            const float *__restrict__ fac32,
                                                            int64_t off0,
                                                            const double *__restrict__ mu,
                                                            float *__restrict__ s32) {
  const int lane = threadIdx.x & 63;
  const FactorSlot &f = fs[0];
  const int rank = f.rank;
  const int r0 = ((int)blockIdx.x * kWavesPerBlock + uniform(threadIdx.x / kWave)) * 32;
  const int q0 = blockIdx.y * 32;
  if (r0 >= rank) return;
  const float *arow[2];
  const double *bcol[2];
  bool aok[2], bok[2];
  for (int h = 0; h < 2; ++h) {
    const int r = r0 + 16 * h + (lane & 15), q = q0 + 16 * h + (lane & 15);
    aok[h] = r < rank;
    bok[h] = q < n_free;
    arow[h] = fac32 + (f.u_off - off0) + (int64_t)(aok[h] ? r : 0) * f.rows;
    bcol[h] = mu + 3 * meta[free_ids[bok[h] ? q : 0]].t0;
  }
  TileTN32 tile;
  mfma_tile_tn32(arow, aok, bcol, bok, f.rows, tile);
  const float *sig = fac32 + (f.sig_off - off0);
  for (int ia = 0; ia < 2; ++ia)
    for (int jb = 0; jb < 2; ++jb)
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + 16 * ia + 4 * (lane >> 4) + v, q = q0 + 16 * jb + (lane & 15);
        if (r < rank && q < n_free) s32[meta[free_ids[q]].s0 + r] = tile.acc[ia][jb][v] / sig[r];
      }
}

// FP32 proxy strengths of every free sphere: str32 = V_0 s32 (contact-free
// spheres have proxies only).
__global__ __launch_bounds__(kBlock) void k_pinv_shared_v32(const int32_t *__restrict__ free_ids,
                                                            int32_t n_free,
                                                            const SphereMeta *__restrict__ meta,
                                                            const FactorSlot *__restrict__ fs,
                                                            const float *__restrict__ fac32,
                                                            int64_t off0,
                                                            const float *__restrict__ s32,
                                                            float *__restrict__ str32) {
  const int lane = threadIdx.x & 63;
  const FactorSlot &f = fs[0];
  const int rows = f.cols;
  const int r0 = ((int)blockIdx.x * kWavesPerBlock + uniform(threadIdx.x / kWave)) * 32;
  const int q0 = blockIdx.y * 32;
  if (r0 >= rows) return;
  const float *arow[2], *bcol[2];
  bool aok[2], bok[2];
  for (int h = 0; h < 2; ++h) {
    const int r = r0 + 16 * h + (lane & 15), q = q0 + 16 * h + (lane & 15);
    aok[h] = r < rows;
    bok[h] = q < n_free;
    arow[h] = fac32 + (f.vt_off - off0) + (int64_t)(aok[h] ? r : 0) * f.cols;
    bcol[h] = s32 + meta[free_ids[bok[h] ? q : 0]].s0;
  }
  TileTN32 tile;
  mfma_tile_tn32(arow, aok, bcol, bok, f.rank, tile);
  for (int ia = 0; ia < 2; ++ia)
    for (int jb = 0; jb < 2; ++jb)
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + 16 * ia + 4 * (lane >> 4) + v, q = q0 + 16 * jb + (lane & 15);
        if (r < rows && q < n_free) {
          const SphereMeta &m = meta[free_ids[q]];
          str32[3 * (m.k0[0] + r / 3) + r % 3] = tile.acc[ia][jb][v];
        }
      }
}

}  // namespace

hipError_t launch_pinv_shared32(const int32_t *free_ids, int32_t n_free, int32_t rank, int32_t cols,
                                const SphereMeta *meta, const FactorSlot *fs, const float *fac32,
                                int64_t off0, const double *mu, float *s32, float *str32,
                                hipStream_t s) {
  if (n_free <= 0 || rank <= 0) return hipSuccess;
  const unsigned qt = (unsigned)((n_free + 31) / 32);
  const unsigned gu = (unsigned)(((rank + 31) / 32 + kWavesPerBlock - 1) / kWavesPerBlock);
  const unsigned gv = (unsigned)(((cols + 31) / 32 + kWavesPerBlock - 1) / kWavesPerBlock);
  hipLaunchKernelGGL(k_pinv_shared_u32, dim3(gu, qt), dim3(kBlock), 0, s, free_ids, n_free, meta, fs,
                     fac32, off0, mu, s32);
  hipLaunchKernelGGL(k_pinv_shared_v32, dim3(gv, qt), dim3(kBlock), 0, s, free_ids, n_free, meta, fs,
                     fac32, off0, s32, str32);
  return hipGetLastError();
}

hipError_t launch_pinv_shared(const int32_t *free_ids, int32_t n_free, int32_t rank, int32_t cols,
                              const SphereMeta *meta, const FactorSlot *fs, const double *fac,
                              const double *mu, double *sbuf, double *lam, double dscale,
                              hipStream_t s) {
  if (n_free <= 0 || rank <= 0) return hipSuccess;
  const unsigned qt = (unsigned)((n_free + 31) / 32);
  const unsigned gu = (unsigned)(((rank + 31) / 32 + kWavesPerBlock - 1) / kWavesPerBlock);
  const unsigned gv = (unsigned)(((cols + 31) / 32 + kWavesPerBlock - 1) / kWavesPerBlock);
  hipLaunchKernelGGL(k_pinv_shared_u, dim3(gu, qt), dim3(kBlock), 0, s, free_ids, n_free, meta, fs, fac,
                     mu, sbuf);
  hipLaunchKernelGGL(k_pinv_shared_v, dim3(gv, qt), dim3(kBlock), 0, s, free_ids, n_free, meta, fs, fac,
                     sbuf, lam, dscale);
  return hipGetLastError();
}

}  // namespace smfs
