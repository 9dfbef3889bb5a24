// C-ABI of libsmfs: problem lifecycle, workspace layout, the one-body
// preconditioned product (Section 2.2), setup of the self-block factors
// (rocSOLVER thin SVD with relative truncation, Section 5) and a
// device-resident GMRES with classical Gram-Schmidt applied twice.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace smfs {

namespace {
thread_local std::string g_err;
constexpr double kPi = 3.14159265358979323846;
constexpr int kTileTargets = 64 * kDirectTpl;   // targets per wave tile
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Source splits of the direct sum: enough blocks (about 32768, i.e. 128 per
// CU; measured best among 8192/16384/32768) to keep every SIMD busy to the
// end of the launch and balance the tail, while each split still streams at
// least 64 sources (small problems, e.g. two spheres with 1320 sources,
// would otherwise run on one wave per tile).
int32_t choose_splits(int64_t n_tiles, int64_t S) {
  const int64_t blocks = std::max<int64_t>(1, (n_tiles + 3) / 4);
  static const int64_t target = [] {
    const char *e = std::getenv("SMFS_DIRECT_BLOCKS");
    return e ? std::max<int64_t>(256, std::atoll(e)) : (int64_t)32768;
  }();
  int64_t sp = (target + blocks - 1) / blocks;
  sp = std::min<int64_t>(sp, std::max<int64_t>(1, S / 64));
  sp = std::max<int64_t>(1, std::min<int64_t>(sp, 64));
  return (int32_t)sp;
}

int64_t free_tiles(int64_t n) { return (n + kTileTargets - 1) / kTileTargets; }

}  // namespace

int32_t direct_splits(int64_t n_tiles, int64_t S) { return choose_splits(n_tiles, S); }

void set_error(const std::string &msg) { g_err = msg; }

bool valid_precision(int p) {
  return p == SMFS_FP64 || p == SMFS_MIXED || p == SMFS_MIXED_FAR || p == SMFS_MIXED_EQ;
}
bool is_mixed(int p) { return p == SMFS_MIXED || p == SMFS_MIXED_FAR || p == SMFS_MIXED_EQ; }
// The equivalent-source far field has contact-free spheres to serve.
bool eq_enabled(const Problem &pb) { return pb.n_eq > 0 && pb.n_free > 0; }

// Tiles of the FP64 direct sums: tt consecutive targets each, whatever
// sphere they belong to, as (first sphere, first target, count, last
// sphere); only the last tile is short.
void build_tiles(const Problem &pb, std::vector<int4> &tiles, int tt) {
  tiles.clear();
  for (int64_t t0 = 0; t0 < pb.T; t0 += tt) {
    const int64_t tc = std::min<int64_t>(tt, pb.T - t0);
    tiles.push_back(make_int4(pb.tsph[t0], (int)t0, (int)tc, pb.tsph[t0 + tc - 1]));
  }
}

// One-sphere tiles, (k, t0, count, k): the FP32 far-field sum (its
// coordinates are relative to the tile's sphere centre) and the block sum
// over many right-hand sides (whose accumulators leave no room for the
// masked pass of a tile across spheres).
void build_sphere_tiles(const Problem &pb, std::vector<int4> &tiles, int tt) {
  tiles.clear();
  for (int k = 0; k < pb.P; ++k) {
    const int64_t t0 = pb.toff[k], M = pb.toff[k + 1] - pb.toff[k];
    for (int64_t o = 0; o < M; o += tt)
      tiles.push_back(make_int4(k, (int)(t0 + o), (int)std::min<int64_t>(tt, M - o), k));
  }
}

// Assign (or only measure) the workspace regions.  Returns bytes needed.
size_t workspace_layout(Problem &pb, bool assign) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const int64_t T = pb.T, S = pb.S, C = pb.C;
  const int P = pb.P;
  const size_t o_tgt = take(sizeof(double) * 3 * T);
  const size_t o_sw = take(sizeof(double) * T);
  const size_t o_tsph = take(sizeof(int32_t) * T);
  const size_t o_src = take(sizeof(double) * 3 * S);
  const size_t o_lam = take(sizeof(double) * 3 * S);
  const size_t o_chk = take(sizeof(double) * 3 * C);
  const size_t o_csph = take(sizeof(int32_t) * C);
  const size_t o_meta = take(sizeof(SphereMeta) * P);
  const size_t o_fs = take(sizeof(FactorSlot) * pb.factors.size());
  std::vector<int4> tiles, stiles;
  build_tiles(pb, tiles, kTileTargets);
  build_sphere_tiles(pb, stiles, kTileTargets);
  const size_t o_tiles = take(sizeof(int4) * tiles.size());
  const size_t o_stiles = take(sizeof(int4) * stiles.size());
  int64_t cols_total = 0;
  for (int k = 0; k < P; ++k) cols_total += pb.factors[pb.fid_of[k]].cols;
  const size_t o_s = take(sizeof(double) * cols_total);
  const size_t o_ut = take(sizeof(RowTask) * cols_total);
  const size_t o_vt = take(sizeof(RowTask) * cols_total);
  int64_t btasks = 0;
  for (int k = 0; k < P; ++k) btasks += (pb.factors[pb.fid_of[k]].cols + 31) / 32;
  const size_t o_bu = take(sizeof(int4) * std::max<int64_t>(1, btasks));
  const size_t o_bv = take(sizeof(int4) * std::max<int64_t>(1, btasks));
  const int32_t sp_t = choose_splits((int64_t)tiles.size(), S);
  const int32_t sp_c = choose_splits(free_tiles(C), S);
  int32_t n_free = 0;
  for (int k = 0; k < P; ++k) n_free += pb.contacts[k].empty() ? 1 : 0;
  const bool eq = pb.prm.eq_points > 0 && n_free > 0;
  // with the equivalent-source far field, one more slice for the near proxies
  const int64_t part = std::max<int64_t>(3 * T * (sp_t + (eq ? 1 : 0)), 3 * C * sp_c);
  const size_t o_part = take(sizeof(double) * part);
  // mixed precision: FP32 coordinates/strengths of proxies, FP32 partials
  const int64_t nprox = pb.nb[0];
  const int32_t sp32 = n_free > 0 ? std::min<int32_t>(choose_splits((int64_t)stiles.size(),
                                                                   (int64_t)n_free * pb.prm.n_proxy),
                                                      std::max(1, n_free)) : 0;
  const int32_t ne = eq ? pb.prm.eq_points : 0;
  const int32_t sp_eq = eq ? std::min<int32_t>(choose_splits((int64_t)tiles.size(), (int64_t)n_free * ne),
                                               std::max(1, n_free)) : 0;
  pb.n_eq = ne;
  if (eq) build_near_lists(pb, pb.prm.eq_separation * pb.a);
  const size_t o_eqE = take(sizeof(double) * std::max<int64_t>(1, (int64_t)9 * ne * pb.prm.n_proxy));
  const size_t o_eqq = take(sizeof(float) * std::max<int64_t>(1, (int64_t)3 * ne * n_free));
  const size_t o_eqpt = take(sizeof(float) * std::max<int64_t>(1, (int64_t)3 * ne));
  const size_t o_noff = take(sizeof(int32_t) * (P + 1));
  const size_t o_nidx = take(sizeof(int32_t) * std::max<size_t>(1, eq ? pb.near_idx.size() : 0));
  const size_t o_tgt32 = take(sizeof(float) * 3 * T);
  const size_t o_src32 = take(sizeof(float) * 3 * nprox);
  const size_t o_str32 = take(sizeof(float) * 3 * nprox);
  const size_t o_part32 = take(sizeof(float) * 3 * T * std::max(std::max(sp32, sp_eq), 1));
  const size_t o_s32 = take(sizeof(float) * cols_total);
  const size_t o_free = take(sizeof(int32_t) * std::max(1, P));
  const size_t o_cen = take(sizeof(double) * 3 * P);
  const size_t o_rng = take(sizeof(SrcRange) * (2 * (P + 8)));
  const FactorSlot &f0 = pb.factors[0];
  const int64_t fac32_elems = f0.rep >= 0 ? (int64_t)f0.rows * f0.cols + (int64_t)f0.cols * f0.cols + f0.cols : 0;
  const size_t o_fac32 = take(sizeof(float) * std::max<int64_t>(1, fac32_elems));
  // Krylov basis (restart + 1 vectors) and work vectors
  // vectors of the mobility system (3 T + 6 P) fit in every Krylov slot
  const int64_t ld = ((3 * T + 6 * (int64_t)P + 31) / 32) * 32;
  const int32_t m = std::max(1, pb.prm.gmres_restart);
  const size_t o_kry = take(sizeof(double) * ld * (m + 1));
  const size_t o_vec = take(sizeof(double) * ld * 9);
  const int32_t nch = mdot_chunks(3 * T + 6 * (int64_t)P);
  const int64_t red = 2 * (int64_t)nch * (m + 2) + 6 * (m + 2) + 1024 + 64;
  const size_t o_red = take(sizeof(double) * red);
  // factors: slots of equal shape are consecutive with a uniform stride so
  // that one strided-batched SVD can write a whole group in place
  const size_t o_fac = off;
  std::vector<int> order;
  for (size_t f = 0; f < pb.factors.size(); ++f)
    if (pb.factors[f].rep >= 0) order.push_back((int)f);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    const FactorSlot &a = pb.factors[x], &b = pb.factors[y];
    return a.rows != b.rows ? a.rows < b.rows : a.cols < b.cols;
  });
  auto slot_elems = [](const FactorSlot &fs) {
    int64_t e = (int64_t)fs.rows * fs.cols + (int64_t)fs.cols * fs.cols + fs.cols;
    return (e + 31) / 32 * 32;
  };
  int64_t fac_elems = 0;
  for (int f : order) fac_elems += slot_elems(pb.factors[f]);
  const size_t fbytes = sizeof(double) * fac_elems;
  take(fbytes);
  if (assign) {
    char *b = pb.ws;
    pb.d_tgt = (double *)(b + o_tgt);
    pb.d_sw = (double *)(b + o_sw);
    pb.d_tsph = (int32_t *)(b + o_tsph);
    pb.d_src = (double *)(b + o_src);
    pb.d_lamhat = (double *)(b + o_lam);
    pb.d_chk = (double *)(b + o_chk);
    pb.d_csph = (int32_t *)(b + o_csph);
    pb.d_meta = (SphereMeta *)(b + o_meta);
    pb.d_fslots = (FactorSlot *)(b + o_fs);
    pb.d_tiles = (int4 *)(b + o_tiles);
    pb.d_stiles = (int4 *)(b + o_stiles);
    pb.d_s = (double *)(b + o_s);
    pb.d_utask = (RowTask *)(b + o_ut);
    pb.d_vtask = (RowTask *)(b + o_vt);
    pb.d_btask_u = (int4 *)(b + o_bu);
    pb.d_btask_v = (int4 *)(b + o_bv);
    pb.cols_total = cols_total;
    pb.d_part = (double *)(b + o_part);
    pb.d_kry = (double *)(b + o_kry);
    pb.d_vec = (double *)(b + o_vec);
    pb.d_red = (double *)(b + o_red);
    pb.d_fac = (double *)(b + o_fac);
    pb.d_tgt32 = (float *)(b + o_tgt32);
    pb.d_src32 = (float *)(b + o_src32);
    pb.d_str32 = (float *)(b + o_str32);
    pb.d_part32 = (float *)(b + o_part32);
    pb.d_s32 = (float *)(b + o_s32);
    pb.d_free = (int32_t *)(b + o_free);
    pb.d_centers = (double *)(b + o_cen);
    pb.d_ranges = (SrcRange *)(b + o_rng);
    pb.d_fac32 = (float *)(b + o_fac32);
    pb.n_free = n_free;
    pb.n_splits32 = sp32;
    pb.d_eqE = (double *)(b + o_eqE);
    pb.d_eqq32 = (float *)(b + o_eqq);
    pb.d_eqpt32 = (float *)(b + o_eqpt);
    pb.d_near_off = (int32_t *)(b + o_noff);
    pb.d_near_idx = (int32_t *)(b + o_nidx);
    pb.n_splits_eq = sp_eq;
    pb.eq_ready = false;
    pb.tiles = tiles;
    pb.n_tiles = (int64_t)tiles.size();
    pb.stiles = stiles;
    pb.n_stiles = (int64_t)stiles.size();
    pb.n_splits = sp_t;
    pb.n_splits_chk = sp_c;
    pb.part_cap = part;
    pb.kry_ld = ld;
    pb.kry_vecs = m + 1;
    pb.red_cap = red;
    // factor offsets (elements from d_fac), grouped by shape
    for (auto &fs : pb.factors) fs.u_off = fs.vt_off = fs.sig_off = 0;
    int64_t e = 0;
    for (int f : order) {
      FactorSlot &fs = pb.factors[f];
      fs.u_off = e;
      fs.vt_off = e + (int64_t)fs.rows * fs.cols;
      fs.sig_off = fs.vt_off + (int64_t)fs.cols * fs.cols;
      e += slot_elems(fs);
    }
  }
  pb.factor_bytes = fbytes;
  return off;
}

int upload_tables(Problem &pb, hipStream_t s) {
  const int P = pb.P;
  std::vector<double> sw(pb.T);
  for (int64_t i = 0; i < pb.T; ++i) sw[i] = pb.prm.left_weights ? std::sqrt(pb.tw[i]) : 1.0;
  pb.meta.assign(P, SphereMeta{});
  for (int k = 0; k < P; ++k) {
    SphereMeta &m = pb.meta[k];
    m.t0 = pb.toff[k];
    m.M = (int32_t)(pb.toff[k + 1] - pb.toff[k]);
    m.N = 0;
    for (int b = 0; b < kBlocks; ++b) {
      m.k0[b] = pb.koff[b][k];
      m.kn[b] = (int32_t)(pb.koff[b][k + 1] - pb.koff[b][k]);
      m.N += m.kn[b];
    }
    m.fid = pb.fid_of[k];
    m.rank = 0;
    m.s0 = 0;
    for (int i = 0; i < 3; ++i) m.c[i] = pb.centers[3 * k + i];
  }
  SMFS_HIP(hipMemcpyAsync(pb.d_tgt, pb.tgt.data(), 8 * pb.tgt.size(), hipMemcpyHostToDevice, s));
  SMFS_HIP(hipMemcpyAsync(pb.d_sw, sw.data(), 8 * sw.size(), hipMemcpyHostToDevice, s));
  SMFS_HIP(hipMemcpyAsync(pb.d_tsph, pb.tsph.data(), 4 * pb.tsph.size(), hipMemcpyHostToDevice, s));
  SMFS_HIP(hipMemcpyAsync(pb.d_src, pb.src.data(), 8 * pb.src.size(), hipMemcpyHostToDevice, s));
  if (pb.C) {
    SMFS_HIP(hipMemcpyAsync(pb.d_chk, pb.chk.data(), 8 * pb.chk.size(), hipMemcpyHostToDevice, s));
    SMFS_HIP(hipMemcpyAsync(pb.d_csph, pb.csph.data(), 4 * pb.csph.size(), hipMemcpyHostToDevice, s));
  }
  SMFS_HIP(hipMemcpyAsync(pb.d_tiles, pb.tiles.data(), sizeof(int4) * pb.tiles.size(),
                          hipMemcpyHostToDevice, s));
  SMFS_HIP(hipMemcpyAsync(pb.d_stiles, pb.stiles.data(), sizeof(int4) * pb.stiles.size(),
                          hipMemcpyHostToDevice, s));
  // mixed precision: coordinates relative to each sphere's centre in FP32
  std::vector<float> t32(3 * pb.T), s32(3 * pb.nb[0]);
  for (int64_t i = 0; i < pb.T; ++i)
    for (int c = 0; c < 3; ++c) t32[3 * i + c] = (float)(pb.tgt[3 * i + c] - pb.centers[3 * pb.tsph[i] + c]);
  for (int64_t j = 0; j < pb.nb[0]; ++j)
    for (int c = 0; c < 3; ++c) s32[3 * j + c] = (float)(pb.src[3 * j + c] - pb.centers[3 * pb.ssph[j] + c]);
  std::vector<int32_t> free_ids;
  for (int k = 0; k < P; ++k)
    if (pb.contacts[k].empty()) free_ids.push_back(k);
  // source ranges: plain = every block; mixed FP64 = proxies of contact
  // spheres (runs of consecutive spheres) and every image block
  std::vector<SrcRange> rng;
  pb.rng_total_plain = 0;
  for (int b = 0; b < kBlocks; ++b)
    if (pb.nb[b] > 0) {
      rng.push_back(SrcRange{(int32_t)pb.koff[b][0], (int32_t)pb.koff[b][P], b, 0});
      pb.rng_total_plain += pb.nb[b];
    }
  pb.n_rng_plain = (int32_t)rng.size();
  pb.rng_total_mixed = 0;
  for (int k = 0; k < P;) {
    if (pb.contacts[k].empty()) { ++k; continue; }
    int e = k;
    while (e < P && !pb.contacts[e].empty()) ++e;
    rng.push_back(SrcRange{(int32_t)pb.koff[0][k], (int32_t)pb.koff[0][e], 0, 0});
    pb.rng_total_mixed += pb.koff[0][e] - pb.koff[0][k];
    k = e;
  }
  for (int b = 1; b < kBlocks; ++b)
    if (pb.nb[b] > 0) {
      rng.push_back(SrcRange{(int32_t)pb.koff[b][0], (int32_t)pb.koff[b][P], b, 0});
      pb.rng_total_mixed += pb.nb[b];
    }
  pb.n_rng_mixed = (int32_t)rng.size() - pb.n_rng_plain;
  SMFS_HIP(hipMemcpyAsync(pb.d_centers, pb.centers.data(), 8 * pb.centers.size(), hipMemcpyHostToDevice, s));
  SMFS_HIP(hipMemcpyAsync(pb.d_tgt32, t32.data(), 4 * t32.size(), hipMemcpyHostToDevice, s));
  if (!s32.empty())
    SMFS_HIP(hipMemcpyAsync(pb.d_src32, s32.data(), 4 * s32.size(), hipMemcpyHostToDevice, s));
  if (!free_ids.empty())
    SMFS_HIP(hipMemcpyAsync(pb.d_free, free_ids.data(), 4 * free_ids.size(), hipMemcpyHostToDevice, s));
  SMFS_HIP(hipMemcpyAsync(pb.d_ranges, rng.data(), sizeof(SrcRange) * rng.size(), hipMemcpyHostToDevice, s));
  std::vector<float> eqpt;
  if (eq_enabled(pb)) {
    std::vector<double> pts;
    spiral_points(pb.n_eq, pb.prm.eq_radius * pb.a, pts);
    eqpt.assign(pts.begin(), pts.end());
    SMFS_HIP(hipMemcpyAsync(pb.d_eqpt32, eqpt.data(), 4 * eqpt.size(), hipMemcpyHostToDevice, s));
    SMFS_HIP(hipMemcpyAsync(pb.d_near_off, pb.near_off.data(), 4 * pb.near_off.size(), hipMemcpyHostToDevice, s));
    if (!pb.near_idx.empty())
      SMFS_HIP(hipMemcpyAsync(pb.d_near_idx, pb.near_idx.data(), 4 * pb.near_idx.size(), hipMemcpyHostToDevice,
                              s));
  }
  SMFS_HIP(hipStreamSynchronize(s));
  return rank_tables(pb, s);
}

// (Re)build the rank-dependent tables: s offsets and the row tasks of the
// pseudo-inverse apply, then upload meta and factor slots.
int rank_tables(Problem &pb, hipStream_t s) {
  // row tasks of contact spheres first, then of contact-free spheres, so
  // that the FP64 tasks of a mixed-precision product are a prefix
  std::vector<RowTask> ut, vt;
  int64_t s0 = 0;
  for (int k = 0; k < pb.P; ++k) {
    SphereMeta &m = pb.meta[k];
    const FactorSlot &f = pb.factors[m.fid];
    m.rank = f.rank;
    m.s0 = s0;
    s0 += f.cols;
  }
  for (int pass = 0; pass < 2; ++pass) {
    for (int k = 0; k < pb.P; ++k) {
      if ((pass == 0) == pb.contacts[k].empty()) continue;
      const FactorSlot &f = pb.factors[pb.meta[k].fid];
      if (f.rank <= 0) continue;
      for (int j = 0; j < f.rank; ++j) ut.push_back(RowTask{k, j});
      for (int i = 0; i < f.cols; ++i) vt.push_back(RowTask{k, i});
    }
    if (pass == 0) {
      pb.n_utask_c = (int64_t)ut.size();
      pb.n_vtask_c = (int64_t)vt.size();
    }
  }
  pb.n_utask = (int64_t)ut.size();
  pb.n_vtask = (int64_t)vt.size();
  // 64-row tiles of the block (many right-hand sides) apply
  std::vector<int4> bu, bv;
  for (int k = 0; k < pb.P; ++k) {
    const FactorSlot &f = pb.factors[pb.meta[k].fid];
    if (f.rank <= 0) continue;
    for (int j = 0; j < f.rank; j += 64) bu.push_back(int4{k, j, 0, 0});
    for (int i = 0; i < f.cols; i += 64) bv.push_back(int4{k, i, 0, 0});
  }
  pb.n_btask_u = (int64_t)bu.size();
  pb.n_btask_v = (int64_t)bv.size();
  // FP32 copy of the shared contact-free factor (mixed precision)
  pb.fac32_ready = false;
  const FactorSlot &f0 = pb.factors[0];
  if (f0.rep >= 0 && f0.rank > 0) {
    const int64_t e = (int64_t)f0.rows * f0.cols + (int64_t)f0.cols * f0.cols + f0.cols;
    SMFS_HIP(launch_to_f32(e, pb.d_fac + f0.u_off, pb.d_fac32, s));
    pb.fac32_ready = true;
  }
  SMFS_HIP(hipMemcpyAsync(pb.d_meta, pb.meta.data(), sizeof(SphereMeta) * pb.P, hipMemcpyHostToDevice, s));
  SMFS_HIP(hipMemcpyAsync(pb.d_fslots, pb.factors.data(), sizeof(FactorSlot) * pb.factors.size(),
                          hipMemcpyHostToDevice, s));
  if (!ut.empty())
    SMFS_HIP(hipMemcpyAsync(pb.d_utask, ut.data(), sizeof(RowTask) * ut.size(), hipMemcpyHostToDevice, s));
  if (!vt.empty())
    SMFS_HIP(hipMemcpyAsync(pb.d_vtask, vt.data(), sizeof(RowTask) * vt.size(), hipMemcpyHostToDevice, s));
  if (!bu.empty())
    SMFS_HIP(hipMemcpyAsync(pb.d_btask_u, bu.data(), sizeof(int4) * bu.size(), hipMemcpyHostToDevice, s));
  if (!bv.empty())
    SMFS_HIP(hipMemcpyAsync(pb.d_btask_v, bv.data(), sizeof(int4) * bv.size(), hipMemcpyHostToDevice, s));
  SMFS_HIP(hipStreamSynchronize(s));
  bool ready = true;
  for (int k = 0; k < pb.P; ++k)
    if (pb.meta[k].rank <= 0) ready = false;
  pb.factors_ready = ready;
  return SMFS_OK;
}

// ---------------------------------------------------------------------------
// Building blocks of the product.

// lambda = B^+ mu for every sphere, FP64 (n_u, n_v limit the task lists:
// the contact-sphere prefix in a mixed-precision product).
int free_transform64(Problem &pb, const double *mu, double *lam, double dscale, hipStream_t s);

int transform_tasks(Problem &pb, const double *mu, double *lam, int64_t n_u, int64_t n_v,
                    double dscale, hipStream_t s) {
  SMFS_HIP(launch_pinv_u(pb.d_utask, n_u, pb.d_meta, pb.d_fslots, pb.d_fac, mu, pb.d_s, s));
  SMFS_HIP(launch_pinv_v(pb.d_vtask, n_v, pb.d_meta, pb.d_fslots, pb.d_fac, pb.d_s, lam, dscale, s));
  return SMFS_OK;
}

// FP64 lambda = B^+ mu for every sphere: contact spheres by per-row GEMV,
// the contact-free spheres through the shared factor as one MFMA GEMM pair.
int transform64(Problem &pb, const double *mu, double *lam, double dscale, hipStream_t s) {
  int rc = transform_tasks(pb, mu, lam, pb.n_utask_c, pb.n_vtask_c, dscale, s);
  if (rc) return rc;
  return free_transform64(pb, mu, lam, dscale, s);
}

// The contact-free spheres only (shared factor, MFMA).
int free_transform64(Problem &pb, const double *mu, double *lam, double dscale, hipStream_t s) {
  const FactorSlot &f0 = pb.factors[0];
  if (pb.n_free > 0 && f0.rep >= 0)
    SMFS_HIP(launch_pinv_shared(pb.d_free, pb.n_free, f0.rank, f0.cols, pb.d_meta, pb.d_fslots, pb.d_fac,
                                mu, pb.d_s, lam, dscale, s));
  return SMFS_OK;
}

// physical strengths lambda = B^+ mu
int transform(Problem &pb, const double *mu, double *lam, hipStream_t s) {
  return transform64(pb, mu, lam, 1.0, s);
}

DirectArgs direct_args(Problem &pb, const double *str, bool mixed) {
  DirectArgs a;
  a.tiles = pb.d_tiles;
  a.tsph = pb.d_tsph;
  a.n_tiles = pb.n_tiles;
  a.tgt = pb.d_tgt;
  a.T = pb.T;
  a.src = pb.d_src;
  a.str = str;
  a.meta = pb.d_meta;
  a.ranges = mixed ? pb.d_ranges + pb.n_rng_plain : pb.d_ranges;
  a.n_ranges = mixed ? pb.n_rng_mixed : pb.n_rng_plain;
  a.range_total = mixed ? pb.rng_total_mixed : pb.rng_total_plain;
  a.dscale = 2.0 * pb.prm.mu;
  a.n_splits = pb.n_splits;
  a.part = pb.d_part;
  return a;
}

// The FP32 far field of the contact-free proxies (mixed precision).
Far32Args far32_args(Problem &pb) {
  Far32Args f;
  f.tiles = pb.d_stiles;
  f.n_tiles = pb.n_stiles;
  f.tgt32 = pb.d_tgt32;
  f.src32 = pb.d_src32;
  f.str32 = pb.d_str32;
  f.free_ids = pb.d_free;
  f.n_free = pb.n_free;
  f.n_proxy = pb.prm.n_proxy;
  f.n_splits = pb.n_splits32;
  f.T = pb.T;
  f.part32 = pb.d_part32;
  f.centers = pb.d_centers;
  return f;
}

// Event pool for smfs_profile: returns the index of a recorded event.
int record_event(Problem &pb, hipStream_t s, size_t &idx) {
  if (pb.ev_used == pb.ev_pool.size()) {
    hipEvent_t e;
    SMFS_HIP(hipEventCreate(&e));
    pb.ev_pool.push_back(e);
  }
  idx = pb.ev_used++;
  SMFS_HIP(hipEventRecord(pb.ev_pool[idx], s));
  return SMFS_OK;
}

// y = G_hat mu.  FP64: every sphere's pseudo-inverse and every off-sphere
// pair in FP64.  Mixed: contact-free spheres (shared factor) go through the
// FP32 pseudo-inverse and the FP32 far-field kernel; contact spheres, with
// their image lines, stay FP64 throughout.
// y = G_hat mu with the equivalent-source far field (SMFS_MIXED_EQ): FP64
// strengths of every sphere; equivalent strengths of the contact-free
// spheres; the FP64 sum over contact spheres' sources (images included),
// the FP64 sum over each target sphere's near contact-free proxies (one
// more partial slice), the FP32 sum over every other contact-free sphere's
// equivalent sources; one epilogue.
int apply_eq(Problem &pb, const double *mu, double *y, hipStream_t s) {
  if (!pb.eq_ready) {
    set_error("SMFS_MIXED_EQ product before smfs_setup_far_field");
    return SMFS_E_STATE;
  }
  size_t e[6] = {0, 0, 0, 0, 0, 0};
  int rc;
  if (pb.prof && (rc = record_event(pb, s, e[0]))) return rc;
  if ((rc = transform64(pb, mu, pb.d_lamhat, 2.0 * pb.prm.mu, s))) return rc;
  if (pb.prof && (rc = record_event(pb, s, e[1]))) return rc;
  SMFS_HIP(launch_eq_strengths(pb.d_eqE, 3 * pb.n_eq, 3 * pb.prm.n_proxy, pb.d_lamhat, pb.d_meta, pb.d_free,
                               pb.n_free, pb.d_eqq32, s));
  if (pb.prof && (rc = record_event(pb, s, e[2]))) return rc;
  DirectArgs a = direct_args(pb, pb.d_lamhat, true);
  SMFS_HIP(launch_direct_f64(a, s));
  if (pb.prof && (rc = record_event(pb, s, e[3]))) return rc;
  NearArgs n;
  n.d = a;
  n.tiles = pb.d_stiles;
  n.n_tiles = pb.n_stiles;
  n.free_ids = pb.d_free;
  n.near_off = pb.d_near_off;
  n.near_idx = pb.d_near_idx;
  n.out = pb.d_part + 3 * pb.T * (int64_t)pb.n_splits;
  SMFS_HIP(launch_near_f64(n, s));
  if (pb.prof && (rc = record_event(pb, s, e[4]))) return rc;
  EqArgs f;
  f.tiles = pb.d_tiles;
  f.n_tiles = pb.n_tiles;
  f.tsph = pb.d_tsph;
  f.tgt = pb.d_tgt;
  f.eqpt32 = pb.d_eqpt32;
  f.q32 = pb.d_eqq32;
  f.centers = pb.d_centers;
  f.free_ids = pb.d_free;
  f.near_off = pb.d_near_off;
  f.near_idx = pb.d_near_idx;
  f.n_free = pb.n_free;
  f.n_eq = pb.n_eq;
  f.n_splits = pb.n_splits_eq;
  f.T = pb.T;
  f.part32 = pb.d_part32;
  SMFS_HIP(launch_far_eq_f32(f, s));
  if (pb.prof && (rc = record_event(pb, s, e[5]))) return rc;
  if (pb.prof) {
    pb.ev_pinv.emplace_back(e[0], e[1]);
    pb.ev_eqq.emplace_back(e[1], e[2]);
    pb.ev_mixed64.emplace_back(e[2], e[3]);
    pb.ev_eqnear.emplace_back(e[3], e[4]);
    pb.ev_eqfar.emplace_back(e[4], e[5]);
  }
  SMFS_HIP(launch_reduce_epilogue(3 * pb.T, pb.n_splits + 1, pb.d_part, pb.n_splits_eq, pb.d_part32, mu, pb.d_sw,
                                  1.0 / (8.0 * kPi * pb.prm.mu), y, s));
  return SMFS_OK;
}

int apply(Problem &pb, const double *mu, double *y, int precision, hipStream_t s) {
  if (precision == SMFS_MIXED_EQ) {
    if (pb.prm.eq_points <= 0) {
      set_error("SMFS_MIXED_EQ needs eq_points > 0");
      return SMFS_E_INVALID_ARG;
    }
    // without contact-free spheres nothing is approximated: the FP64 product
    if (eq_enabled(pb)) return apply_eq(pb, mu, y, s);
    precision = SMFS_FP64;
  }
  const bool mixed = is_mixed(precision) && pb.n_free > 0 && pb.fac32_ready;
  size_t e0 = 0, e1 = 0, e2 = 0, e3 = 0;
  int rc;
  if (pb.prof && (rc = record_event(pb, s, e0))) return rc;
  // dipole strengths pre-multiplied by 2 mu for the direct-sum kernel
  const double ds = 2.0 * pb.prm.mu;
  if (!mixed) {
    rc = transform64(pb, mu, pb.d_lamhat, ds, s);
  } else if (precision == SMFS_MIXED_FAR) {
    // FP64 strengths everywhere, then an FP32 copy of the proxy strengths
    // (block 0) for the far-field kernel
    rc = transform64(pb, mu, pb.d_lamhat, ds, s);
    SMFS_HIP(launch_to_f32(3 * pb.nb[0], pb.d_lamhat, pb.d_str32, s));
  } else {
    // contact spheres in FP64; the contact-free ones by the FP32 GEMMs of
    // the shared factor (its FP32 copy holds factor 0 only)
    rc = transform_tasks(pb, mu, pb.d_lamhat, pb.n_utask_c, pb.n_vtask_c, ds, s);
    const FactorSlot &f0 = pb.factors[0];
    SMFS_HIP(launch_pinv_shared32(pb.d_free, pb.n_free, f0.rank, f0.cols, pb.d_meta, pb.d_fslots,
                                  pb.d_fac32, f0.u_off, mu, pb.d_s32, pb.d_str32, s));
  }
  if (rc) return rc;
  if (pb.prof && (rc = record_event(pb, s, e1))) return rc;
  DirectArgs a = direct_args(pb, pb.d_lamhat, mixed);
  SMFS_HIP(launch_direct_f64(a, s));
  if (pb.prof && (rc = record_event(pb, s, e2))) return rc;
  int32_t ns32 = 0;
  if (mixed) {
    SMFS_HIP(launch_far_f32(far32_args(pb), s));
    ns32 = pb.n_splits32;
    if (pb.prof && (rc = record_event(pb, s, e3))) return rc;
  }
  if (pb.prof) {
    pb.ev_pinv.emplace_back(e0, e1);
    if (mixed) pb.ev_mixed64.emplace_back(e1, e2), pb.ev_far32.emplace_back(e2, e3);
    else pb.ev_direct.emplace_back(e1, e2);
  }
  SMFS_HIP(launch_reduce_epilogue(3 * pb.T, pb.n_splits, pb.d_part, ns32, mixed ? pb.d_part32 : nullptr,
                                  mu, pb.d_sw, 1.0 / (8.0 * kPi * pb.prm.mu), y, s));
  return SMFS_OK;
}

// u = sum over every source at n free points (chunked to the part buffer).
int eval_points(Problem &pb, const double *lam, int64_t n, const double *x, double *u, hipStream_t s) {
  if (n <= 0) return SMFS_OK;
  const int32_t sp = pb.n_splits_chk;
  int64_t cap = pb.part_cap / (3 * sp);   // points whose partial sums fit
  if (cap >= kTileTargets) cap = cap / kTileTargets * kTileTargets;
  if (cap < 1) { set_error("partial-sum buffer too small"); return SMFS_E_NOMEM; }
  for (int64_t o = 0; o < n; o += cap) {
    const int64_t cnt = std::min(cap, n - o);
    DirectArgs a = direct_args(pb, lam, false);
    a.tiles = nullptr;
    a.n_tiles = free_tiles(cnt);
    a.tgt = x + 3 * o;
    a.n_splits = sp;
    a.T = cnt;
    SMFS_HIP(launch_direct_f64(a, s));
    SMFS_HIP(launch_reduce_epilogue(3 * cnt, sp, pb.d_part, 0, nullptr, nullptr, nullptr,
                                    1.0 / (8.0 * kPi * pb.prm.mu), u + 3 * o, s));
  }
  return SMFS_OK;
}

// ---------------------------------------------------------------------------
// GMRES on G_hat mu = b with x0 = 0, restarted every gmres_restart steps,
// Givens rotations on the host.  Arnoldi by classical Gram-Schmidt applied
// twice in its delayed form: step j computes V^T [q_j, A q_j] in one pass
// over the basis, which gives both the second-pass coefficients s of q_j
// (whose first pass ran in step j-1) and the first-pass coefficients z of
// A q_j; one more pass then reorthogonalises q_j and projects A q_j.  The
// column of the Hessenberg matrix that q_j closes is corrected for the
// change of q_j (H[:, j-1] += H[j, j-1] s, H[j, j-1] *= nu) and only then
// rotated, so the residual estimate trails the newest product by one step.
// In exact arithmetic this is the same basis and Hessenberg matrix as
// Gram-Schmidt applied twice, with two passes over the basis per step
// instead of four.

struct GmresStats {
  int iterations = 0;           // Krylov dimension reached (summed over cycles)
  int applies = 0;              // products with the operator
  int check_applies = 0;        // products spent on true-residual checks
  double rel_residual = 0.0;
  bool converged = false;
  bool stagnated = false;       // stopped: the true residual no longer falls
  int true_checks = 0;          // true-residual checks made
  int floor_it = -1;            // iteration of the smallest true residual checked
  double floor_rel = -1.0;      // that residual (relative)
};

// The true-residual guard starts once the recursive estimate is below this
// level: above it the estimate and the true residual agree to many digits.
constexpr double kGuardStart = 1e-3;

// y = A x for the system being solved (precision of the product given).
using Operator = std::function<int(const double *, double *, int)>;

constexpr int32_t kUpdParts = 1024;   // partial sums of the fused update

int gmres(Problem &pb, int64_t n, const Operator &op, const double *b, double *x, GmresStats &st,
          int precision, double tol, int max_it, int check_every, hipStream_t s) {
  const int64_t ld = pb.kry_ld;
  const int m = pb.kry_vecs - 1;
  double *V = pb.d_kry;
  double *w = pb.d_vec;           // scratch vector
  double *r = pb.d_vec + ld;      // residual
  // true-residual guard: trial iterate, its residual, best iterate so far
  double *xt = pb.d_vec + 6 * ld, *wt = pb.d_vec + 7 * ld, *xbest = pb.d_vec + 8 * ld;
  const int32_t nch = mdot_chunks(n);
  double *part = pb.d_red;                                // 2 nch (m + 2)
  double *hd = part + 2 * (int64_t)nch * (m + 2);         // V^T q_j | V^T w, 2 (m + 2)
  double *coef = hd + 2 * (m + 2);                        // [1/nu, gam, nu] of the step
  double *cf = coef + 2 * (m + 2);                        // solution coefficients, m + 2
  double *scal = cf + (m + 2);                            // [0] norm of p, [1] other norms
  double *upart = scal + 8;                               // kUpdParts
  // The host keeps up to kAhead steps behind the device: each step's dot
  // products, its (nu, gam) and the norm of the previous p go to a pinned
  // ring slot, and the Hessenberg column and Givens rotations of a step are
  // formed from its slot once its copy has landed.  Steps enqueued past the
  // one that stops the cycle only touch basis vectors beyond the solution.
  constexpr int kAhead = 2, kRing = kAhead + 2;
  const size_t slot_n = 2 * (size_t)(m + 2) + 8;
  double *hpin = nullptr;
  // kRing step slots, then the guard's coefficients (m + 2) and its norm
  SMFS_HIP(hipHostMalloc((void **)&hpin, sizeof(double) * (slot_n * kRing + m + 3), hipHostMallocDefault));
  double *hchk = hpin + slot_n * kRing;
  std::vector<hipEvent_t> ev(kRing, nullptr);
  struct Free {
    double *p;
    std::vector<hipEvent_t> *e;
    ~Free() {
      if (p) (void)hipHostFree(p);
      for (hipEvent_t x : *e)
        if (x) (void)hipEventDestroy(x);
    }
  } guard{hpin, &ev};
  for (auto &e : ev) SMFS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  // Hraw: the Hessenberg matrix as built (column-major, m+1 rows); R: its
  // rotated copy for the least-squares problem
  std::vector<double> Hraw((size_t)(m + 1) * m, 0.0), R((size_t)(m + 1) * m, 0.0), cs(m), sn(m),
      g(m + 1), y(m), cvec(m + 1);
  auto Hc = [&](std::vector<double> &M, int row, int col) -> double & { return M[(size_t)col * (m + 1) + row]; };

  SMFS_HIP(launch_fill(n, 0.0, x, s));
  SMFS_HIP(launch_norm2(b, n, part, nch, scal + 1, s));
  SMFS_HIP(hipMemcpyAsync(hpin, scal + 1, 8, hipMemcpyDeviceToHost, s));
  SMFS_HIP(hipStreamSynchronize(s));
  const double bnorm = hpin[0];
  st = GmresStats{};
  if (bnorm == 0.0) {
    st.converged = true;
    return SMFS_OK;
  }
  SMFS_HIP(hipMemcpyAsync(r, b, 8 * n, hipMemcpyDeviceToDevice, s));
  double beta = bnorm;
  int enq_applies = 0;   // products enqueued (st.applies counts those the solve used)
  double prev_check = -1.0;   // true residual at the previous in-cycle check
  int last_check_it = 0;
  bool use_best = false;      // the solve ends on xbest rather than on x + V y
  // Records a true residual tr of the iterate in xt (or in x when at_x);
  // keeps the best iterate in xbest.
  auto record_true = [&](double tr, bool at_x) -> int {
    ++st.true_checks;
    if (st.floor_rel < 0 || tr < st.floor_rel) {
      st.floor_rel = tr;
      st.floor_it = st.iterations;
      SMFS_HIP(hipMemcpyAsync(xbest, at_x ? x : xt, 8 * n, hipMemcpyDeviceToDevice, s));
    }
    return SMFS_OK;
  };
  while (true) {
    // V[0] = r / beta (final: it needs no second pass)
    SMFS_HIP(hipMemcpyAsync(V, r, 8 * n, hipMemcpyDeviceToDevice, s));
    SMFS_HIP(launch_norm_scale(V, n, part, nch, scal + 1, scal + 2, s));
    std::fill(g.begin(), g.end(), 0.0);
    std::fill(Hraw.begin(), Hraw.end(), 0.0);
    g[0] = beta;
    int jdone = 0;   // columns of H final in this cycle
    bool stop = false, cycle_end = false;
    int next = 0;    // next step to process on the host
    int last_j = -1; // the step that closes the cycle, once enqueued
    std::vector<int> applies_at(m + 2, 0);
    // host side of step jp (the arithmetic of the synchronous form)
    auto process = [&](int jp) -> int {
      double *slot = hpin + (size_t)(jp % kRing) * slot_n;
      SMFS_HIP(hipEventSynchronize(ev[jp % kRing]));
      const int nv = jp + 1;
      const double *sv = slot, *zv = slot + nv;   // V^T q_j, V^T w
      const double pnorm = slot[2 * (m + 2)], inv_nu = slot[2 * (m + 2) + 1],
                   gam = slot[2 * (m + 2) + 2], nu = slot[2 * (m + 2) + 3];
      (void)inv_nu;
      if (jp > 0) {
        // finalise column jp-1 (q_jp reorthogonalised), rotate it
        Hc(Hraw, jp, jp - 1) = pnorm;   // ||p|| of the previous step
        for (int i = 0; i < jp; ++i) Hc(Hraw, i, jp - 1) += Hc(Hraw, jp, jp - 1) * sv[i];
        Hc(Hraw, jp, jp - 1) *= nu;
        const int c = jp - 1;
        for (int i = 0; i <= jp; ++i) Hc(R, i, c) = Hc(Hraw, i, c);
        double *col = &R[(size_t)c * (m + 1)];
        for (int i = 0; i < c; ++i) {
          const double t = cs[i] * col[i] + sn[i] * col[i + 1];
          col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
          col[i] = t;
        }
        const double den = std::hypot(col[c], col[c + 1]);
        cs[c] = den > 0 ? col[c] / den : 1.0;
        sn[c] = den > 0 ? col[c + 1] / den : 0.0;
        col[c] = den;
        col[c + 1] = 0.0;
        g[c + 1] = -sn[c] * g[c];
        g[c] = cs[c] * g[c];
        jdone = jp;
        ++st.iterations;
        if (pb.prm.progress > 0 && st.iterations % pb.prm.progress == 0) {
          std::fprintf(stderr, "[smfs] GMRES iteration %d, residual estimate %.3e\n", st.iterations,
                       std::fabs(g[c + 1]) / bnorm);
          std::fflush(stderr);
        }
        st.applies = applies_at[jp];
        st.rel_residual = std::fabs(g[c + 1]) / bnorm;
        if (st.rel_residual <= tol) { st.converged = true; stop = true; return SMFS_OK; }
        if (nu == 0.0) { stop = true; return SMFS_OK; }   // q_j lies in the span: exact solution
        // Guard: every check_every iterations once the estimate is small,
        // form the iterate, apply the FP64 operator and take the true
        // residual.
        // Rounding of the truncated pseudo-inverses leaves a floor that the
        // recursive estimate does not see; once the true residual stops
        // falling (less than halved since the last check) while the
        // estimate runs ahead of it by a factor of ten, the solve stops on
        // the best iterate checked.
        if (check_every > 0 && st.rel_residual <= kGuardStart &&
            st.iterations - last_check_it >= check_every) {
          last_check_it = st.iterations;
          const int nj = jdone;
          for (int i = nj - 1; i >= 0; --i) {
            double t = g[i];
            for (int c2 = i + 1; c2 < nj; ++c2) t -= Hc(R, i, c2) * hchk[c2];
            hchk[i] = t / Hc(R, i, i);
          }
          SMFS_HIP(hipMemcpyAsync(cf, hchk, 8 * (size_t)nj, hipMemcpyHostToDevice, s));
          SMFS_HIP(hipMemcpyAsync(xt, x, 8 * n, hipMemcpyDeviceToDevice, s));
          SMFS_HIP(launch_combine(V, ld, nj, cf, xt, n, s));
          // the check is an FP64 product whatever the Krylov products are:
          // in a mixed solve the residual of the FP32 far field stalls at
          // its rounding level while the iterate still improves
          int rc = op(xt, wt, SMFS_FP64);
          if (rc) return rc;
          ++st.check_applies;
          SMFS_HIP(launch_sub(n, b, wt, wt, s));
          SMFS_HIP(launch_norm2(wt, n, part, nch, scal + 4, s));
          SMFS_HIP(hipMemcpyAsync(hchk + m + 2, scal + 4, 8, hipMemcpyDeviceToHost, s));
          SMFS_HIP(hipStreamSynchronize(s));
          const double tr = hchk[m + 2] / bnorm;
          if ((rc = record_true(tr, false))) return rc;
          if (tr <= tol) { st.converged = true; stop = use_best = true; return SMFS_OK; }
          if (prev_check > 0 && tr > 0.5 * prev_check && st.rel_residual < 0.1 * tr) {
            st.stagnated = true;
            stop = use_best = true;
            return SMFS_OK;
          }
          prev_check = tr;
        }
        if (jp == last_j) {
          if (st.applies >= max_it) stop = true;
          cycle_end = true;                                // end of the cycle
          return SMFS_OK;
        }
      }
      // column jp of Hraw: c = Hraw[0..jp, 0..jp-1] s, the part of A q_jp
      // carried by the old q_jp
      std::fill(cvec.begin(), cvec.begin() + jp + 1, 0.0);
      for (int k = 0; k < jp; ++k)
        for (int i = 0; i <= k + 1; ++i) cvec[i] += Hc(Hraw, i, k) * sv[k];
      for (int i = 0; i < jp; ++i) Hc(Hraw, i, jp) = (zv[i] - cvec[i]) / nu;
      Hc(Hraw, jp, jp) = (gam - cvec[jp]) / nu;
      return SMFS_OK;
    };
    for (int j = 0; !stop && !cycle_end; ++j) {
      const bool last = j == m || (enq_applies >= max_it && j > 0);
      double *qj = V + (int64_t)j * ld, *wj = V + (int64_t)(j + 1) * ld;
      if (!last) {
        int rc = op(qj, wj, precision);
        if (rc) return rc;
        ++enq_applies;
      }
      applies_at[j] = enq_applies;
      // the slot of step j is free: step j - kRing was processed (the host
      // stays at most kAhead steps behind)
      const int nv = j + 1;
      double *slot = hpin + (size_t)(j % kRing) * slot_n;
      SMFS_HIP(launch_mdot2(V, ld, nv, qj, last ? qj : wj, n, part, nch, hd, s));
      SMFS_HIP(launch_dcgs_coeffs(hd, j, coef, s));
      SMFS_HIP(hipMemcpyAsync(slot, hd, 8 * 2 * (size_t)nv, hipMemcpyDeviceToHost, s));
      SMFS_HIP(hipMemcpyAsync(slot + 2 * (m + 2), scal, 8, hipMemcpyDeviceToHost, s));
      SMFS_HIP(hipMemcpyAsync(slot + 2 * (m + 2) + 1, coef, 8 * 3, hipMemcpyDeviceToHost, s));
      SMFS_HIP(hipEventRecord(ev[j % kRing], s));
      if (last) last_j = j;
      else
        SMFS_HIP(launch_dcgs_update(V, ld, j, hd, hd + nv, qj, wj, coef, n, upart, kUpdParts, scal, s));
      // process what the device has (or must have) finished
      while (next <= j && !stop && !cycle_end &&
             (last || j - next >= kAhead || hipEventQuery(ev[next % kRing]) == hipSuccess)) {
        int rc = process(next);
        if (rc) return rc;
        ++next;
      }
    }
    if (use_best) {   // the guard ended the solve on a checked iterate
      SMFS_HIP(hipMemcpyAsync(x, xbest, 8 * n, hipMemcpyDeviceToDevice, s));
      SMFS_HIP(hipStreamSynchronize(s));
      return SMFS_OK;
    }
    // y = R^-1 g (upper triangular), x += V y
    for (int i = jdone - 1; i >= 0; --i) {
      double t = g[i];
      for (int c = i + 1; c < jdone; ++c) t -= Hc(R, i, c) * y[c];
      y[i] = t / Hc(R, i, i);
    }
    SMFS_HIP(hipMemcpyAsync(cf, y.data(), 8 * jdone, hipMemcpyHostToDevice, s));
    SMFS_HIP(launch_combine(V, ld, jdone, cf, x, n, s));
    SMFS_HIP(hipStreamSynchronize(s));
    if (stop) return SMFS_OK;
    // restart from the true residual (an FP64 product in every mode)
    int rc = op(x, w, SMFS_FP64);
    if (rc) return rc;
    ++st.check_applies;
    enq_applies = st.applies;
    SMFS_HIP(launch_sub(n, b, w, r, s));
    SMFS_HIP(launch_norm2(r, n, part, nch, scal + 1, s));
    SMFS_HIP(hipMemcpyAsync(hpin, scal + 1, 8, hipMemcpyDeviceToHost, s));
    SMFS_HIP(hipStreamSynchronize(s));
    beta = hpin[0];
    if (beta / bnorm <= tol) {
      st.converged = true;
      st.rel_residual = beta / bnorm;
      return SMFS_OK;
    }
    if (check_every > 0) {
      // a restart is a true-residual check: a cycle that brought it no
      // lower than 0.9 of the best seen ends the solve on the best iterate
      const double tr = beta / bnorm, best = st.floor_rel;
      int rc = record_true(tr, true);
      if (rc) return rc;
      if (best > 0 && tr > 0.9 * best) {
        st.stagnated = true;
        st.rel_residual = tr;
        SMFS_HIP(hipMemcpyAsync(x, xbest, 8 * n, hipMemcpyDeviceToDevice, s));
        SMFS_HIP(hipStreamSynchronize(s));
        return SMFS_OK;
      }
    }
  }
}

}  // namespace smfs

using namespace smfs;


extern "C" {

const char *smfs_last_error(void) { return g_err.c_str(); }

int smfs_params_default(smfs_params *p) {
  if (!p) { set_error("null params"); return SMFS_E_INVALID_ARG; }
  std::memset(p, 0, sizeof(*p));
  p->n_proxy = 600;
  p->proxy_radius = 0.7;
  p->n_colloc_base = 780;
  p->n_image = 20;
  p->image_kinds = SMFS_KIND_S | SMFS_KIND_R | SMFS_KIND_D;
  p->image_offset = 0.05;
  p->image_gap_cutoff = 0.2;
  p->near_gap_cutoff = 0.2;
  p->cap_alpha[0] = p->cap_alpha[1] = 6;
  p->cap_beta[0] = kPi / 5.0;
  p->cap_beta[1] = kPi / 60.0;
  p->left_weights = 1;
  p->trunc_rel = 5e-12;
  p->mu = 1.0;
  p->n_check_base = 500;
  p->precision = SMFS_FP64;
  p->gmres_tol = 1e-10;
  p->gmres_max_it = 1000;
  p->gmres_restart = 400;
  p->gmres_check_every = 25;
  p->svd_method = SMFS_SVD_ROCSOLVER;
  p->eq_points = 200;
  p->eq_radius = 1.0;
  p->eq_check_radius = 2.5;
  p->eq_separation = 3.5;
  p->eq_rcond = 1e-12;
  p->progress = 0;
  return SMFS_OK;
}

int smfs_problem_create(const smfs_params *p, int32_t P, const double *centers,
                        const double *radii, smfs_problem **out) {
  if (!p || !centers || !radii || !out || P <= 0) {
    set_error("smfs_problem_create: null argument or P <= 0");
    return SMFS_E_INVALID_ARG;
  }
  *out = nullptr;
  if (p->n_proxy <= 0 || p->n_colloc_base <= 0 || p->gmres_restart > 20000 || !(p->proxy_radius > 0 && p->proxy_radius < 1) ||
      !(p->mu > 0) || !(p->trunc_rel >= 0) || p->gmres_restart <= 0 || p->gmres_max_it <= 0 ||
      p->n_check_base < 0 || p->cap_alpha[0] < 0 || p->cap_alpha[1] < 0 || p->gmres_check_every < 0 ||
      (p->svd_method != SMFS_SVD_JACOBI && p->svd_method != SMFS_SVD_ROCSOLVER) ||
      p->eq_points < 0 || p->eq_points > 4096 || p->progress < 0 ||
      (p->eq_points > 0 && !(p->eq_radius > 0 && p->eq_check_radius > p->eq_radius &&
                             p->eq_separation >= p->eq_check_radius + 1.0 && p->eq_rcond > 0 &&
                             p->eq_rcond < 1)) ||
      !valid_precision(p->precision)) {
    set_error("smfs_problem_create: invalid parameter");
    return SMFS_E_INVALID_ARG;
  }
  if (p->near_gap_cutoff > p->image_gap_cutoff) {
    set_error("smfs_problem_create: near_gap_cutoff above image_gap_cutoff is not supported");
    return SMFS_E_UNSUPPORTED;
  }
  for (int i = 0; i < 3 * P; ++i)
    if (!std::isfinite(centers[i])) {
      set_error("smfs_problem_create: non-finite centre");
      return SMFS_E_INVALID_ARG;
    }
  for (int k = 0; k < P; ++k) {
    if (!(radii[k] > 0) || !std::isfinite(radii[k])) {
      set_error("smfs_problem_create: radius must be positive");
      return SMFS_E_INVALID_ARG;
    }
    if (radii[k] != radii[0]) {
      set_error("smfs_problem_create: spheres of unequal radii are not supported");
      return SMFS_E_UNSUPPORTED;
    }
  }
  smfs_problem *pb = new smfs_problem();
  pb->prm = *p;
  pb->P = P;
  pb->a = radii[0];
  pb->centers.assign(centers, centers + 3 * P);
  int rc = build_geometry(*pb);
  if (rc < 0) { delete pb; return rc; }
  pb->need_bytes = workspace_layout(*pb, false);
  *out = pb;
  return pb->small_gap ? SMFS_GAP_BELOW_VALIDATED : SMFS_OK;
}

void smfs_problem_destroy(smfs_problem *pb) {
  if (!pb) return;
  for (hipEvent_t e : pb->ev_pool) (void)hipEventDestroy(e);
  if (pb->rocblas) rocblas_destroy_handle((rocblas_handle)pb->rocblas);
  delete pb;
}

int smfs_problem_sizes(const smfs_problem *pb, smfs_sizes *s) {
  if (!pb || !s) { set_error("null argument"); return SMFS_E_INVALID_ARG; }
  std::memset(s, 0, sizeof(*s));
  s->P = pb->P;
  s->n_factors = (int32_t)pb->factors.size();
  s->n_contacts = pb->n_contacts;
  s->min_gap_flag = pb->small_gap ? 1 : 0;
  s->T = pb->T;
  s->S = pb->S;
  for (int i = 0; i < 3; ++i) s->n_kind[i] = pb->nk[i];
  s->n_check = pb->C;
  s->workspace_bytes = pb->need_bytes;
  s->factor_bytes = pb->factor_bytes;
  s->svd_sweeps = pb->svd_sweeps;
  if (pb->n_eq > 0) {   // set when the form is on and some sphere is contact-free
    s->eq_far_pairs = pb->pairs_eq_far;
    s->eq_exact_pairs = pb->pairs_eq_exact;
    s->eq_near_spheres = (int64_t)pb->near_idx.size();
  }
  return SMFS_OK;
}

int smfs_export_nodes(const smfs_problem *pb, double *targets, int32_t *target_sphere,
                      double *target_weight, double *sources, int32_t *source_kind,
                      int32_t *source_sphere, double *check, int32_t *check_sphere) {
  if (!pb) { set_error("null problem"); return SMFS_E_INVALID_ARG; }
  if (targets) std::memcpy(targets, pb->tgt.data(), 8 * pb->tgt.size());
  if (target_sphere) std::memcpy(target_sphere, pb->tsph.data(), 4 * pb->tsph.size());
  if (target_weight) std::memcpy(target_weight, pb->tw.data(), 8 * pb->tw.size());
  if (sources) std::memcpy(sources, pb->src.data(), 8 * pb->src.size());
  if (source_kind) std::memcpy(source_kind, pb->skind.data(), 4 * pb->skind.size());
  if (source_sphere) std::memcpy(source_sphere, pb->ssph.data(), 4 * pb->ssph.size());
  if (check) std::memcpy(check, pb->chk.data(), 8 * pb->chk.size());
  if (check_sphere) std::memcpy(check_sphere, pb->csph.data(), 4 * pb->csph.size());
  return SMFS_OK;
}

int smfs_sphere_factor(const smfs_problem *pb, int32_t k, int32_t *fid) {
  if (!pb || !fid || k < 0 || k >= pb->P) { set_error("bad sphere index"); return SMFS_E_INVALID_ARG; }
  *fid = pb->fid_of[k];
  return SMFS_OK;
}

int smfs_factor_info(const smfs_problem *pb, int32_t fid, int32_t *rows, int32_t *cols,
                     int32_t *rank, int32_t *sphere) {
  if (!pb || fid < 0 || fid >= (int32_t)pb->factors.size()) {
    set_error("bad factor id");
    return SMFS_E_INVALID_ARG;
  }
  const FactorSlot &f = pb->factors[fid];
  if (rows) *rows = f.rows;
  if (cols) *cols = f.cols;
  if (rank) *rank = f.rank;
  if (sphere) *sphere = f.rep;
  return SMFS_OK;
}

int smfs_bind(smfs_problem *pb, void *ws, size_t bytes, smfs_stream stream) {
  if (!pb || !ws) { set_error("smfs_bind: null argument"); return SMFS_E_INVALID_ARG; }
  if (bytes < pb->need_bytes) {
    set_error("smfs_bind: workspace of " + std::to_string(bytes) + " bytes, need " +
              std::to_string(pb->need_bytes));
    return SMFS_E_NOMEM;
  }
  if (((uintptr_t)ws) % kAlign) { set_error("smfs_bind: workspace must be 256-byte aligned"); return SMFS_E_INVALID_ARG; }
  pb->ws = (char *)ws;
  pb->ws_bytes = bytes;
  for (auto &f : pb->factors) f.rank = 0;
  workspace_layout(*pb, true);
  int rc = upload_tables(*pb, (hipStream_t)stream);
  if (rc) return rc;
  pb->bound = true;
  return SMFS_OK;
}

}  // extern "C"

namespace smfs {

// Shape groups of the distinct self blocks (consecutive in the workspace,
// see workspace_layout): factor ids sorted by slot, split where the shape
// changes.  Factor 0 is left out when it was imported (skip_shared).
struct ShapeGroup {
  std::vector<int> fids;
  int m = 0, n = 0;
  int64_t stride = 0;      // elements between consecutive slots of the group
  int nb = 1;              // blocks per batched SVD call
};

constexpr int kSvdBatchMax = 32;

std::vector<ShapeGroup> shape_groups(const Problem &pb) {
  std::vector<int> order;
  for (size_t f = 0; f < pb.factors.size(); ++f)
    if (pb.factors[f].rep >= 0 && !(pb.skip_shared && f == 0)) order.push_back((int)f);
  std::sort(order.begin(), order.end(),
            [&](int x, int y) { return pb.factors[x].u_off < pb.factors[y].u_off; });
  std::vector<ShapeGroup> out;
  for (int f : order) {
    const FactorSlot &fs = pb.factors[f];
    if (out.empty() || out.back().m != fs.rows || out.back().n != fs.cols) {
      out.emplace_back();
      out.back().m = fs.rows;
      out.back().n = fs.cols;
    }
    out.back().fids.push_back(f);
  }
  for (ShapeGroup &g : out) {
    // the Jacobi sweeps launch once per round whatever the batch: batches of
    // small blocks up to 256 blocks or 2 GiB of blocks
    int cap = kSvdBatchMax;
    if (pb.prm.svd_method == SMFS_SVD_JACOBI)
      cap = (int)std::max<int64_t>(kSvdBatchMax, std::min<int64_t>(256, ((int64_t)2 << 30) / (8 * (int64_t)g.m * g.n)));
    g.nb = (int)std::min<size_t>((size_t)cap, g.fids.size());
    g.stride = g.fids.size() > 1 ? pb.factors[g.fids[1]].u_off - pb.factors[g.fids[0]].u_off : 0;
  }
  return out;
}

int ensure_rocblas(Problem &pb) {
  if (!pb.rocblas) {
    rocblas_handle h;
    if (rocblas_create_handle(&h) != rocblas_status_success) {
      set_error("rocblas_create_handle failed");
      return SMFS_E_DEVICE;
    }
    pb.rocblas = h;
  }
  return SMFS_OK;
}

// Scratch of one batched SVD call of group g: [SVD work | A copies | E | info].
struct SvdScratch {
  size_t work = 0, a = 0, e = 0, info = 0, total = 0;
};

int svd_scratch_plan(Problem &pb, const ShapeGroup &g, SvdScratch &sc) {
  int rc = ensure_rocblas(pb);
  if (rc) return rc;
  rocblas_handle h = (rocblas_handle)pb.rocblas;
  // size query: nothing runs and no pointer is dereferenced
  double *fake = reinterpret_cast<double *>((uintptr_t)4096);
  rocblas_int *ifake = reinterpret_cast<rocblas_int *>((uintptr_t)4096);
  size_t work = 0;
  if (rocblas_start_device_memory_size_query(h) != rocblas_status_success) {
    set_error("rocblas_start_device_memory_size_query failed");
    return SMFS_E_DEVICE;
  }
  const rocblas_stride st = std::max<int64_t>(g.stride, 1);
  rocblas_status q = rocsolver_dgesvd_strided_batched(
      h, rocblas_svect_singular, rocblas_svect_singular, g.m, g.n, fake, g.m,
      (rocblas_stride)g.m * g.n, fake, st, fake, g.m, st, fake, g.n, st, fake, g.n,
      rocblas_outofplace, ifake, g.nb);
  rocblas_status q2 = rocblas_stop_device_memory_size_query(h, &work);
  if ((q != rocblas_status_success && q != rocblas_status_size_increased &&
       q != rocblas_status_size_unchanged) || q2 != rocblas_status_success) {
    set_error("SVD workspace query failed with status " + std::to_string((int)q));
    return SMFS_E_SVD;
  }
  sc.work = align_up(work);
  sc.a = align_up(sizeof(double) * (size_t)g.m * g.n * g.nb);
  sc.e = align_up(sizeof(double) * (size_t)g.n * g.nb);
  sc.info = align_up(sizeof(rocblas_int) * g.nb);
  sc.total = sc.work + sc.a + sc.e + sc.info;
  return SMFS_OK;
}

int setup_scratch_bytes(Problem &pb, size_t &bytes) {
  bytes = 0;
  for (const ShapeGroup &g : shape_groups(pb)) {
    if (pb.prm.svd_method == SMFS_SVD_JACOBI) {
      int rc = ensure_rocblas(pb);
      if (rc) return rc;
      JacPlan jp;
      if ((rc = jacobi_plan((rocblas_handle)pb.rocblas, g.m, g.n, g.nb, jp))) return rc;
      bytes = std::max(bytes, jp.total);
    } else {
      SvdScratch sc;
      int rc = svd_scratch_plan(pb, g, sc);
      if (rc) return rc;
      bytes = std::max(bytes, sc.total);
    }
  }
  return SMFS_OK;
}

// The device Jacobi SVD of every shape group (B = Q1 R1, R1^T = Q2 R2,
// one-sided Jacobi on R2^T, U = Q1 U_X, V = Q2 J), the blocks assembled
// into the plan's input region.
int setup_factors_jacobi(Problem &pb, char *scratch, size_t scratch_bytes, hipStream_t s) {
  rocblas_handle h = (rocblas_handle)pb.rocblas;
  for (const ShapeGroup &g : shape_groups(pb)) {
    JacPlan jp;
    int rc = jacobi_plan(h, g.m, g.n, g.nb, jp);
    if (rc) return rc;
    if (scratch_bytes < jp.total) {
      set_error("smfs_setup: scratch of " + std::to_string(scratch_bytes) + " bytes, need " +
                std::to_string(jp.total));
      return SMFS_E_NOMEM;
    }
    double *A = (double *)(scratch + jp.work);
    const int m = g.m, n = g.n;
    for (size_t b0 = 0; b0 < g.fids.size(); b0 += g.nb) {
      const int real = (int)std::min<size_t>(g.nb, g.fids.size() - b0);
      std::vector<double *> U(real), V(real), S(real);
      for (int q = 0; q < real; ++q) {
        const FactorSlot &fs = pb.factors[g.fids[b0 + q]];
        const SphereMeta &mk = pb.meta[fs.rep];
        SMFS_HIP(launch_assemble_block(pb.d_tgt, pb.d_sw, pb.d_src, pb.d_meta, fs.rep, mk.M, mk.N,
                                       pb.prm.mu, A + (size_t)q * m * n, s));
        U[q] = pb.d_fac + fs.u_off;
        V[q] = pb.d_fac + fs.vt_off;
        S[q] = pb.d_fac + fs.sig_off;
      }
      JacPlan jr;   // the plan of this call's batch count (no larger than jp)
      if ((rc = jacobi_plan(h, m, n, real, jr))) return rc;
      jr.work = jp.work;   // the same layout start: the input region stays where it was assembled
      std::vector<int> ranks(real, 0);
      int sweeps = 0;
      rc = jacobi_svd_batch(h, jr, scratch, m, n, real, U.data(), V.data(), S.data(), pb.prm.trunc_rel,
                            ranks.data(), &sweeps, s);
      if (rc) return rc;
      pb.svd_sweeps = std::max(pb.svd_sweeps, sweeps);
      for (int q = 0; q < real; ++q) pb.factors[g.fids[b0 + q]].rank = ranks[q];
    }
  }
  (void)rocblas_set_workspace(h, nullptr, 0);
  return rank_tables(pb, s);
}

// Assemble and factor every distinct self block with scratch memory given
// by the caller (no device memory is allocated here: rocSOLVER works in the
// scratch through the handle's user workspace).
int setup_factors(Problem &pb, char *scratch, size_t scratch_bytes, hipStream_t s) {
  int rc = ensure_rocblas(pb);
  if (rc) return rc;
  rocblas_handle h = (rocblas_handle)pb.rocblas;
  rocblas_set_stream(h, s);
  pb.svd_sweeps = 0;
  if (pb.prm.svd_method == SMFS_SVD_JACOBI) return setup_factors_jacobi(pb, scratch, scratch_bytes, s);
  for (const ShapeGroup &g : shape_groups(pb)) {
    SvdScratch sc;
    if ((rc = svd_scratch_plan(pb, g, sc))) return rc;
    if (scratch_bytes < sc.total) {
      set_error("smfs_setup: scratch of " + std::to_string(scratch_bytes) + " bytes, need " +
                std::to_string(sc.total));
      return SMFS_E_NOMEM;
    }
    if (rocblas_set_workspace(h, scratch, sc.work) != rocblas_status_success) {
      set_error("rocblas_set_workspace failed");
      return SMFS_E_DEVICE;
    }
    double *A = (double *)(scratch + sc.work);
    double *E = (double *)(scratch + sc.work + sc.a);
    rocblas_int *info = (rocblas_int *)(scratch + sc.work + sc.a + sc.e);
    const int m = g.m, n = g.n;
    for (size_t b0 = 0; b0 < g.fids.size(); b0 += g.nb) {
      // the last call of a group may be shorter (its scratch need is no larger)
      const int real = (int)std::min<size_t>(g.nb, g.fids.size() - b0);
      for (int q = 0; q < real; ++q) {
        const FactorSlot &fs = pb.factors[g.fids[b0 + q]];
        const SphereMeta &mk = pb.meta[fs.rep];
        SMFS_HIP(launch_assemble_block(pb.d_tgt, pb.d_sw, pb.d_src, pb.d_meta, fs.rep, mk.M, mk.N,
                                       pb.prm.mu, A + (size_t)q * m * n, s));
      }
      const FactorSlot &fb = pb.factors[g.fids[b0]];
      double *U = pb.d_fac + fb.u_off, *VT = pb.d_fac + fb.vt_off, *sig = pb.d_fac + fb.sig_off;
      const rocblas_stride st = std::max<int64_t>(g.stride, 1);
      rocblas_status stt = rocsolver_dgesvd_strided_batched(
          h, rocblas_svect_singular, rocblas_svect_singular, m, n, A, m, (rocblas_stride)m * n, sig,
          st, U, m, st, VT, n, st, E, n, rocblas_outofplace, info, real);
      if (stt != rocblas_status_success) {
        (void)rocblas_set_workspace(h, nullptr, 0);
        set_error("rocsolver_dgesvd_strided_batched failed with status " + std::to_string((int)stt));
        return SMFS_E_SVD;
      }
      std::vector<rocblas_int> hinfo(real);
      std::vector<double> sv((size_t)n * real);
      SMFS_HIP(hipMemcpyAsync(hinfo.data(), info, sizeof(rocblas_int) * real, hipMemcpyDeviceToHost, s));
      for (int q = 0; q < real; ++q)
        SMFS_HIP(hipMemcpyAsync(sv.data() + (size_t)q * n, sig + (size_t)q * g.stride, 8 * (size_t)n,
                                hipMemcpyDeviceToHost, s));
      SMFS_HIP(hipStreamSynchronize(s));
      for (int q = 0; q < real; ++q) {
        const double *sq = sv.data() + (size_t)q * n;
        if (hinfo[q] != 0 || !(sq[0] > 0)) {
          (void)rocblas_set_workspace(h, nullptr, 0);
          set_error("SVD did not converge (info " + std::to_string(hinfo[q]) + ")");
          return SMFS_E_SVD;
        }
        int r = 0;
        while (r < n && sq[r] > pb.prm.trunc_rel * sq[0]) ++r;
        pb.factors[g.fids[b0 + q]].rank = r;
      }
    }
  }
  (void)rocblas_set_workspace(h, nullptr, 0);
  return rank_tables(pb, s);
}

// Scratch regions of the equivalent-source fit (bytes, 256-aligned each):
// rocSOLVER/rocBLAS work, the point sets, K(check, equivalent) (m x n),
// K(check, proxies) (m x cp), sigma, U, V^T, the superdiagonal, info and
// the intermediate product (n x cp); m = 6 n_eq, n = 3 n_eq, cp = 3 N.
struct EqPlan {
  size_t work = 0, pts = 0, kce = 0, kcp = 0, sv = 0, u = 0, vt = 0, e = 0, info = 0, t1 = 0, total = 0;
};

int eq_plan(Problem &pb, EqPlan &q) {
  q = EqPlan{};
  if (!eq_enabled(pb)) return SMFS_OK;
  int rc = ensure_rocblas(pb);
  if (rc) return rc;
  rocblas_handle h = (rocblas_handle)pb.rocblas;
  const int ne = pb.n_eq, nc = 2 * ne, np = pb.prm.n_proxy;
  const int m = 3 * nc, n = 3 * ne, cp = 3 * np;
  double *fake = reinterpret_cast<double *>((uintptr_t)4096);
  size_t w1 = 0, w2 = 0;
  rocblas_start_device_memory_size_query(h);
  rocblas_status q1 = rocsolver_dgesvd(h, rocblas_svect_singular, rocblas_svect_singular, m, n, fake, m, fake, fake,
                                       m, fake, n, fake, rocblas_outofplace, reinterpret_cast<rocblas_int *>(fake));
  rocblas_stop_device_memory_size_query(h, &w1);
  const double one = 1.0, zero = 0.0;
  rocblas_start_device_memory_size_query(h);
  rocblas_status q2 = rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, n, cp, m, &one, fake, m,
                                    fake, m, &zero, fake, n);
  rocblas_stop_device_memory_size_query(h, &w2);
  auto ok = [](rocblas_status x) {
    return x == rocblas_status_success || x == rocblas_status_size_increased || x == rocblas_status_size_unchanged;
  };
  if (!ok(q1) || !ok(q2)) {
    set_error("far-field set-up: workspace query failed");
    return SMFS_E_SVD;
  }
  q.work = align_up(std::max(w1, w2));
  q.pts = align_up(sizeof(double) * 3 * (size_t)(nc + ne + np));
  q.kce = align_up(sizeof(double) * (size_t)m * n);
  q.kcp = align_up(sizeof(double) * (size_t)m * cp);
  q.sv = align_up(sizeof(double) * (size_t)n);
  q.u = align_up(sizeof(double) * (size_t)m * n);
  q.vt = align_up(sizeof(double) * (size_t)n * n);
  q.e = align_up(sizeof(double) * (size_t)n);
  q.info = align_up(sizeof(rocblas_int));
  q.t1 = align_up(sizeof(double) * (size_t)n * cp);
  q.total = q.work + q.pts + q.kce + q.kcp + q.sv + q.u + q.vt + q.e + q.info + q.t1;
  return SMFS_OK;
}

// E = K_ce^+ K_cp for the contact-free proxies (the map from proxy to
// equivalent strengths), into the workspace; the pseudo-inverse keeps the
// singular values of K_ce above eq_rcond sigma_1.
int setup_far_field(Problem &pb, char *scratch, size_t scratch_bytes, hipStream_t s) {
  pb.eq_ready = false;
  if (!eq_enabled(pb)) return SMFS_OK;
  EqPlan q;
  int rc = eq_plan(pb, q);
  if (rc) return rc;
  if (scratch_bytes < q.total) {
    set_error("smfs_setup_far_field: scratch of " + std::to_string(scratch_bytes) + " bytes, need " +
              std::to_string(q.total));
    return SMFS_E_NOMEM;
  }
  rocblas_handle h = (rocblas_handle)pb.rocblas;
  const int ne = pb.n_eq, nc = 2 * ne, np = pb.prm.n_proxy;
  const int m = 3 * nc, n = 3 * ne, cp = 3 * np;
  char *o = scratch;
  char *work = o; o += q.work;
  double *pts = (double *)o; o += q.pts;
  double *Kce = (double *)o; o += q.kce;
  double *Kcp = (double *)o; o += q.kcp;
  double *sv = (double *)o; o += q.sv;
  double *U = (double *)o; o += q.u;
  double *Vt = (double *)o; o += q.vt;
  double *E = (double *)o; o += q.e;
  rocblas_int *info = (rocblas_int *)o; o += q.info;
  double *T1 = (double *)o; o += q.t1;
  // check points, equivalent points, the proxies of a contact-free sphere
  // relative to its centre (host)
  std::vector<double> xc, ye, h_pts;
  spiral_points(nc, pb.prm.eq_check_radius * pb.a, xc);
  spiral_points(ne, pb.prm.eq_radius * pb.a, ye);
  int kf = 0;
  while (!pb.contacts[kf].empty()) ++kf;
  if (pb.koff[0][kf + 1] - pb.koff[0][kf] != np) {
    set_error("far-field set-up: a contact-free sphere without n_proxy proxies");
    return SMFS_E_INVALID_ARG;
  }
  h_pts.insert(h_pts.end(), xc.begin(), xc.end());
  h_pts.insert(h_pts.end(), ye.begin(), ye.end());
  for (int64_t j = pb.koff[0][kf]; j < pb.koff[0][kf + 1]; ++j)
    for (int c = 0; c < 3; ++c) h_pts.push_back(pb.src[3 * j + c] - pb.centers[3 * kf + c]);
  SMFS_HIP(hipMemcpyAsync(pts, h_pts.data(), 8 * h_pts.size(), hipMemcpyHostToDevice, s));
  const double *dxc = pts, *dye = pts + 3 * nc, *dyp = pts + 3 * (nc + ne);
  SMFS_HIP(launch_stokeslet_matrix(dxc, nc, dye, ne, Kce, s));
  SMFS_HIP(launch_stokeslet_matrix(dxc, nc, dyp, np, Kcp, s));
  rocblas_set_stream(h, s);
  if (rocblas_set_workspace(h, work, q.work) != rocblas_status_success) {
    set_error("far-field set-up: rocblas_set_workspace failed");
    return SMFS_E_DEVICE;
  }
  struct Reset {
    rocblas_handle h;
    ~Reset() { (void)rocblas_set_workspace(h, nullptr, 0); }
  } reset{h};
  if (rocsolver_dgesvd(h, rocblas_svect_singular, rocblas_svect_singular, m, n, Kce, m, sv, U, m, Vt, n, E,
                       rocblas_outofplace, info) != rocblas_status_success) {
    set_error("far-field set-up: gesvd failed");
    return SMFS_E_SVD;
  }
  std::vector<double> hs(n);
  rocblas_int hinfo = 0;
  SMFS_HIP(hipMemcpyAsync(hs.data(), sv, 8 * (size_t)n, hipMemcpyDeviceToHost, s));
  SMFS_HIP(hipMemcpyAsync(&hinfo, info, sizeof(rocblas_int), hipMemcpyDeviceToHost, s));
  SMFS_HIP(hipStreamSynchronize(s));
  if (hinfo != 0 || !(hs[0] > 0) || !std::isfinite(hs[0])) {
    set_error("far-field set-up: SVD did not converge");
    return SMFS_E_SVD;
  }
  int r = 0;
  while (r < n && hs[r] > pb.prm.eq_rcond * hs[0]) ++r;
  // T1 = (U_r Sigma_r^-1)^T K_cp (r x cp, ld n), E = V_r T1 (n x cp, ld n)
  SMFS_HIP(launch_scale_cols(U, m, r, sv, s));
  const double one = 1.0, zero = 0.0;
  if (rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, r, cp, m, &one, U, m, Kcp, m, &zero,
                    T1, n) != rocblas_status_success ||
      rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, n, cp, r, &one, Vt, n, T1, n, &zero,
                    pb.d_eqE, n) != rocblas_status_success) {
    set_error("far-field set-up: gemm failed");
    return SMFS_E_DEVICE;
  }
  SMFS_HIP(hipStreamSynchronize(s));
  pb.eq_ready = true;
  return SMFS_OK;
}

}  // namespace smfs

extern "C" {

int smfs_setup_workspace_bytes(smfs_problem *pb, size_t *bytes) {
  if (!pb || !bytes) { set_error("smfs_setup_workspace_bytes: null argument"); return SMFS_E_INVALID_ARG; }
  int rc = setup_scratch_bytes(*pb, *bytes);
  if (rc) return rc;
  EqPlan q;
  if ((rc = eq_plan(*pb, q))) return rc;
  *bytes = std::max(*bytes, q.total);
  return SMFS_OK;
}

int smfs_setup(smfs_problem *pb, void *scratch, size_t scratch_bytes, smfs_stream stream) {
  if (!pb || !pb->bound) { set_error("smfs_setup: problem not bound"); return SMFS_E_STATE; }
  if (!scratch || ((uintptr_t)scratch) % kAlign) {
    set_error("smfs_setup: scratch must be a 256-byte aligned device pointer");
    return SMFS_E_INVALID_ARG;
  }
  int rc = setup_factors(*pb, (char *)scratch, scratch_bytes, (hipStream_t)stream);
  if (rc) return rc;
  return setup_far_field(*pb, (char *)scratch, scratch_bytes, (hipStream_t)stream);
}

int smfs_far_field_workspace_bytes(smfs_problem *pb, size_t *bytes) {
  if (!pb || !bytes) { set_error("smfs_far_field_workspace_bytes: null argument"); return SMFS_E_INVALID_ARG; }
  EqPlan q;
  int rc = eq_plan(*pb, q);
  *bytes = q.total;
  return rc;
}

int smfs_setup_far_field(smfs_problem *pb, void *scratch, size_t scratch_bytes, smfs_stream stream) {
  if (!pb || !pb->bound) { set_error("smfs_setup_far_field: problem not bound"); return SMFS_E_STATE; }
  if (!eq_enabled(*pb)) return SMFS_OK;
  if (!scratch || ((uintptr_t)scratch) % kAlign) {
    set_error("smfs_setup_far_field: scratch must be a 256-byte aligned device pointer");
    return SMFS_E_INVALID_ARG;
  }
  return setup_far_field(*pb, (char *)scratch, scratch_bytes, (hipStream_t)stream);
}

int smfs_import_factor(smfs_problem *pb, int32_t fid, int32_t rank, const double *U,
                       const double *sigma, const double *V, smfs_stream stream) {
  if (!pb || !pb->bound) { set_error("smfs_import_factor: problem not bound"); return SMFS_E_STATE; }
  if (fid < 0 || fid >= (int32_t)pb->factors.size() || !U || !sigma || !V) {
    set_error("smfs_import_factor: bad argument");
    return SMFS_E_INVALID_ARG;
  }
  FactorSlot &fs = pb->factors[fid];
  if (fs.rep < 0 || rank <= 0 || rank > fs.cols) {
    set_error("smfs_import_factor: rank out of range or unused factor");
    return SMFS_E_INVALID_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  SMFS_HIP(hipMemcpyAsync(pb->d_fac + fs.u_off, U, 8 * (size_t)fs.rows * rank, hipMemcpyHostToDevice, s));
  SMFS_HIP(hipMemcpyAsync(pb->d_fac + fs.sig_off, sigma, 8 * (size_t)rank, hipMemcpyHostToDevice, s));
  SMFS_HIP(hipMemcpy2DAsync(pb->d_fac + fs.vt_off, 8 * (size_t)fs.cols, V, 8 * (size_t)rank,
                            8 * (size_t)rank, fs.cols, hipMemcpyHostToDevice, s));
  fs.rank = rank;
  return rank_tables(*pb, s);
}


int smfs_apply(smfs_problem *pb, const double *mu, double *y, int32_t precision, smfs_stream stream) {
  SMFS_READY(pb);
  if (!mu || !y || mu == y) { set_error("smfs_apply: bad vectors"); return SMFS_E_INVALID_ARG; }
  if (!valid_precision(precision)) { set_error("bad precision"); return SMFS_E_INVALID_ARG; }
  return apply(*pb, mu, y, precision, (hipStream_t)stream);
}

int smfs_transform(smfs_problem *pb, const double *mu, double *lam, smfs_stream stream) {
  SMFS_READY(pb);
  if (!mu || !lam) { set_error("smfs_transform: null vector"); return SMFS_E_INVALID_ARG; }
  return transform(*pb, mu, lam, (hipStream_t)stream);
}

int smfs_rhs(smfs_problem *pb, const double *rbm, double *b, smfs_stream stream) {
  if (!pb || !pb->bound) { set_error("problem not bound"); return SMFS_E_STATE; }
  if (!rbm || !b) { set_error("smfs_rhs: null vector"); return SMFS_E_INVALID_ARG; }
  SMFS_HIP(launch_rhs(pb->T, pb->d_tgt, pb->d_tsph, pb->d_sw, pb->d_meta, rbm, b, (hipStream_t)stream,
                      &pb->bg));
  return SMFS_OK;
}

int smfs_set_background(smfs_problem *pb, const double *U, const double *L) {
  if (!pb) { set_error("null problem"); return SMFS_E_INVALID_ARG; }
  BgFlow bg{};
  double lmax = 0.0;
  for (int q = 0; q < 3; ++q) bg.U[q] = U ? U[q] : 0.0;
  for (int q = 0; q < 9; ++q) {
    bg.L[q] = L ? L[q] : 0.0;
    lmax = std::max(lmax, std::fabs(bg.L[q]));
  }
  for (int q = 0; q < 3; ++q)
    if (!std::isfinite(bg.U[q])) { set_error("background flow: non-finite U"); return SMFS_E_INVALID_ARG; }
  for (int q = 0; q < 9; ++q)
    if (!std::isfinite(bg.L[q])) { set_error("background flow: non-finite gradient"); return SMFS_E_INVALID_ARG; }
  // a linear flow solves the homogeneous Stokes equations only if it is
  // divergence-free
  if (std::fabs(bg.L[0] + bg.L[4] + bg.L[8]) > 1e-12 * lmax) {
    set_error("background flow: velocity gradient is not trace-free");
    return SMFS_E_INVALID_ARG;
  }
  bg.on = (U != nullptr || L != nullptr) ? 1 : 0;
  pb->bg = bg;
  return SMFS_OK;
}

int smfs_force_torque(smfs_problem *pb, const double *lam, double *ft, smfs_stream stream) {
  if (!pb || !pb->bound) { set_error("problem not bound"); return SMFS_E_STATE; }
  if (!lam || !ft) { set_error("smfs_force_torque: null vector"); return SMFS_E_INVALID_ARG; }
  SMFS_HIP(launch_force_torque(pb->P, pb->d_meta, pb->d_src, lam, ft, (hipStream_t)stream));
  return SMFS_OK;
}

int smfs_eval_velocity(smfs_problem *pb, const double *lam, int64_t n, const double *x, double *u,
                       smfs_stream stream) {
  if (!pb || !pb->bound) { set_error("problem not bound"); return SMFS_E_STATE; }
  if (n < 0 || (n > 0 && (!lam || !x || !u))) { set_error("smfs_eval_velocity: bad argument"); return SMFS_E_INVALID_ARG; }
  return eval_points(*pb, lam, n, x, u, (hipStream_t)stream);
}

int64_t smfs_pairs_per_apply(const smfs_problem *pb) { return pb ? pb->pairs_per_apply : 0; }

int smfs_set_solver(smfs_problem *pb, int32_t precision, double gmres_tol, int32_t gmres_max_it) {
  if (!pb || !valid_precision(precision) || !(gmres_tol > 0) ||
      gmres_max_it <= 0) {
    set_error("smfs_set_solver: bad argument");
    return SMFS_E_INVALID_ARG;
  }
  pb->prm.precision = precision;
  pb->prm.gmres_tol = gmres_tol;
  pb->prm.gmres_max_it = gmres_max_it;
  return SMFS_OK;
}

int smfs_profile(smfs_problem *pb, int32_t enable) {
  if (!pb) { set_error("null problem"); return SMFS_E_INVALID_ARG; }
  if (enable) {
    pb->ev_used = 0;
    pb->ev_direct.clear();
    pb->ev_pinv.clear();
    pb->ev_mixed64.clear();
    pb->ev_far32.clear();
    pb->ev_bdirect.clear();
    pb->ev_bpinv.clear();
    pb->ev_eqfar.clear();
    pb->ev_eqnear.clear();
    pb->ev_eqq.clear();
    pb->prof_nrhs = 0;
  }
  pb->prof = enable != 0;
  return SMFS_OK;
}

int smfs_profile_read(smfs_problem *pb, smfs_kernel_stats *st) {
  if (!pb || !st) { set_error("null argument"); return SMFS_E_INVALID_ARG; }
  std::memset(st, 0, sizeof(*st));
  auto total = [pb](const std::vector<std::pair<size_t, size_t>> &ev, double &sum) -> int {
    for (auto &pr : ev) {
      float ms = 0.f;
      SMFS_HIP(hipEventSynchronize(pb->ev_pool[pr.second]));
      SMFS_HIP(hipEventElapsedTime(&ms, pb->ev_pool[pr.first], pb->ev_pool[pr.second]));
      sum += ms;
    }
    return (int)SMFS_OK;
  };
  int rc;
  if ((rc = total(pb->ev_direct, st->direct_ms)) || (rc = total(pb->ev_pinv, st->pinv_ms)) ||
      (rc = total(pb->ev_mixed64, st->mixed64_ms)) || (rc = total(pb->ev_far32, st->far32_ms)) ||
      (rc = total(pb->ev_bdirect, st->bdirect_ms)) || (rc = total(pb->ev_bpinv, st->bpinv_ms)) ||
      (rc = total(pb->ev_eqfar, st->eq_far_ms)) || (rc = total(pb->ev_eqnear, st->eq_near_ms)) ||
      (rc = total(pb->ev_eqq, st->eq_strength_ms)))
    return rc;
  st->eq_launches = (int64_t)pb->ev_eqfar.size();
  st->eq_far_flops = 28.0 * pb->pairs_eq_far;
  {
    // near proxies: every target sphere against its near list's proxies
    double nearp = 0.0;
    for (int k = 0; k < pb->P && !pb->near_off.empty(); ++k)
      nearp += (double)(pb->toff[k + 1] - pb->toff[k]) * (pb->near_off[k + 1] - pb->near_off[k]) *
               pb->prm.n_proxy;
    st->eq_near_flops = 28.0 * nearp;
  }
  st->mixed64_launches = (int64_t)pb->ev_mixed64.size();
  st->direct_launches = (int64_t)pb->ev_direct.size();
  st->pinv_launches = (int64_t)pb->ev_pinv.size();
  st->far32_launches = (int64_t)pb->ev_far32.size();
  st->bdirect_launches = (int64_t)pb->ev_bdirect.size();
  st->bpinv_launches = (int64_t)pb->ev_bpinv.size();
  st->bnrhs = pb->prof_nrhs;
  st->far32_flops = 28.0 * pb->pairs_f32;
  st->mixed64_flops = 28.0 * (pb->pairs_kind[0] - pb->pairs_f32) + 25.0 * pb->pairs_kind[1] +
                      30.0 * pb->pairs_kind[2];
  st->direct_flops = 28.0 * pb->pairs_kind[0] + 25.0 * pb->pairs_kind[1] + 30.0 * pb->pairs_kind[2];
  // block direct sum: geometry once per pair (10, 10, 12 flops), then
  // 18, 15, 18 flops per pair and right-hand side (sums to 28, 25, 30)
  const double q = pb->prof_nrhs;
  st->bdirect_flops = (10.0 + 18.0 * q) * pb->pairs_kind[0] + (10.0 + 15.0 * q) * pb->pairs_kind[1] +
                      (12.0 + 18.0 * q) * pb->pairs_kind[2];
  double gemm = 0.0;
  for (int k = 0; k < pb->P; ++k) {
    const FactorSlot &f = pb->factors[pb->fid_of[k]];
    gemm += 2.0 * q * ((double)f.rows * f.rank + (double)f.cols * f.rank);
  }
  st->bpinv_flops = gemm;
  // minimal traffic of the FP64 apply: every contact sphere's factors, the
  // shared factor once, mu read and lambda written
  double bytes = 8.0 * (3.0 * pb->T + 3.0 * pb->S);
  for (size_t f = 0; f < pb->factors.size(); ++f) {
    const FactorSlot &fs = pb->factors[f];
    if (fs.rep >= 0) bytes += 8.0 * ((double)fs.rows * fs.rank + (double)fs.cols * fs.rank);
  }
  st->pinv_bytes = bytes;
  return SMFS_OK;
}

}  // extern "C"

namespace smfs {

// Mobility operator (augmented system in (mu, V)): top rows G_hat mu -
// W Psi V, bottom rows the scaled forces and torques of lambda = B^+ mu.
int apply_mobility(Problem &pb, const double *x, double *y, int precision, hipStream_t s) {
  const int64_t n = 3 * pb.T;
  int rc = apply(pb, x, y, precision, s);
  if (rc) return rc;
  const bool mixed = precision == SMFS_MIXED && pb.n_free > 0 && pb.fac32_ready;
  if (mixed) {  // FP64 strengths of the contact-free spheres for their forces
    rc = free_transform64(pb, x, pb.d_lamhat, 2.0 * pb.prm.mu, s);
    if (rc) return rc;
  }
  SMFS_HIP(launch_rigid(pb.T, pb.d_tgt, pb.d_tsph, pb.d_sw, pb.d_meta, x + n, -1.0, 1.0, y, s));
  const double sF = 1.0 / (6.0 * kPi * pb.prm.mu * pb.a), sT = 1.0 / (8.0 * kPi * pb.prm.mu * pb.a * pb.a * pb.a);
  SMFS_HIP(launch_force_torque(pb.P, pb.d_meta, pb.d_src, pb.d_lamhat, y + n, s, sF, sT));
  return SMFS_OK;
}

struct SolveStats {
  int iterations = 0, refinements = 0;
  int applies = 0;              // products with the operator, in the solve's precision
  int applies64 = 0;            // FP64 true-residual products
  bool converged = false;       // the FP64 true residual meets gmres_tol
  bool stagnated = false;       // stopped at the true-residual floor above gmres_tol
  int true_checks = 0, floor_it = -1;
  double floor_rel = -1.0;
  double rel_residual = 0.0, res_norm = 0.0, rhs_norm = 0.0;
};

// Status of a finished solve: OK only when the FP64 true residual meets the
// tolerance; STAGNATED when it stopped falling above it (the guard, or the
// recursive estimate met the tolerance while the true residual did not);
// NOT_CONVERGED when the iteration limit came first.
int solve_status(const SolveStats &ss) {
  if (ss.converged) return SMFS_OK;
  return ss.stagnated ? SMFS_STAGNATED : SMFS_NOT_CONVERGED;
}

// GMRES on A x = b (x0 = 0), then the true residual in FP64 and up to two
// refinement sweeps on it: GMRES on A d = r, x += d.  Mixed products refine
// whenever the FP64 residual misses the tolerance; FP64 products once the
// iteration stopped above it (the estimate or the guard ended a Krylov
// process whose rounding left a residual floor; a fresh process on the
// residual starts below that floor).  A sweep that leaves a larger true
// residual is taken back.
int solve_system(Problem &pb, int64_t n, const Operator &op, const double *b, double *x,
                 int precision, SolveStats &ss, hipStream_t s) {
  const int64_t ld = pb.kry_ld;
  const double tol = pb.prm.gmres_tol;
  const int every = pb.prm.gmres_check_every;
  GmresStats st;
  int rc = gmres(pb, n, op, b, x, st, precision, tol, pb.prm.gmres_max_it, every, s);
  if (rc) return rc;
  ss = SolveStats{};
  ss.iterations = st.iterations;
  ss.applies = st.applies;
  ss.applies64 = st.check_applies;
  ss.rel_residual = st.rel_residual;
  ss.true_checks = st.true_checks;
  ss.floor_it = st.floor_it;
  ss.floor_rel = st.floor_rel;
  // the estimate met the tolerance, or the guard stopped the iteration
  bool stopped = st.converged || st.stagnated;
  double *w = pb.d_vec, *r = pb.d_vec + ld, *rr = pb.d_vec + 4 * ld, *d = pb.d_vec + 5 * ld;
  const int32_t nch = mdot_chunks(n);
  double *scal = pb.d_red + pb.red_cap - 8;
  double hres[2] = {0, 0}, prev_res[2] = {0, 0};
  double prev_true = -1.0;
  while (true) {
    rc = op(x, w, SMFS_FP64);
    if (rc) return rc;
    ++ss.applies64;
    SMFS_HIP(launch_sub(n, b, w, r, s));
    SMFS_HIP(launch_norm2(r, n, pb.d_red, nch, scal, s));
    SMFS_HIP(launch_norm2(b, n, pb.d_red, nch, scal + 1, s));
    SMFS_HIP(hipMemcpyAsync(hres, scal, 16, hipMemcpyDeviceToHost, s));
    SMFS_HIP(hipStreamSynchronize(s));
    const double true_rel = hres[1] > 0 ? hres[0] / hres[1] : 0.0;
    if (ss.refinements > 0 && !(true_rel <= prev_true)) {
      // the last sweep did not lower the true residual: take it back
      SMFS_HIP(launch_axpby(n, -1.0, d, 1.0, x, s));
      hres[0] = prev_res[0];
      hres[1] = prev_res[1];
      ss.converged = prev_true <= tol;
      ss.stagnated = !ss.converged;
      break;
    }
    ss.converged = true_rel <= tol;
    ss.stagnated = !ss.converged && stopped;
    if (ss.converged || ss.refinements >= 2 || ss.applies >= pb.prm.gmres_max_it ||
        (!is_mixed(precision) && !ss.stagnated))
      break;
    prev_true = true_rel;
    prev_res[0] = hres[0];
    prev_res[1] = hres[1];
    SMFS_HIP(hipMemcpyAsync(rr, r, 8 * n, hipMemcpyDeviceToDevice, s));
    const double tol_d = std::min(0.5, std::max(tol, tol / true_rel));
    GmresStats sd;
    rc = gmres(pb, n, op, rr, d, sd, precision, tol_d, pb.prm.gmres_max_it - ss.applies, every, s);
    if (rc) return rc;
    ss.iterations += sd.iterations;
    ss.applies += sd.applies;
    ss.applies64 += sd.check_applies;
    ss.true_checks += sd.true_checks;
    stopped = sd.converged || sd.stagnated;
    SMFS_HIP(launch_axpby(n, 1.0, d, 1.0, x, s));
    ++ss.refinements;
  }
  ss.res_norm = hres[0];
  ss.rhs_norm = hres[1];
  return SMFS_OK;
}

// lambda, forces/torques, max |lambda| and the check-point residual for
// the rigid motions rbm [dev].
int post_process(Problem &pb, const double *x, const double *rbm, smfs_out *out, double *stats,
                 hipStream_t s) {
  double *lam = out->lambda ? out->lambda : pb.d_lamhat;
  int rc = transform(pb, x, lam, s);
  if (rc) return rc;
  double *scal = pb.d_red + pb.red_cap - 8;
  if (out->ft) SMFS_HIP(launch_force_torque(pb.P, pb.d_meta, pb.d_src, lam, out->ft, s));
  SMFS_HIP(launch_absmax(3 * pb.S, lam, scal + 2, s));
  if (out->u_check && pb.C) {
    rc = eval_points(pb, lam, pb.C, pb.d_chk, out->u_check, s);
    if (rc) return rc;
    SMFS_HIP(launch_residual_stats(pb.C, pb.d_chk, pb.d_csph, pb.d_meta, rbm, out->u_check, 1e-3,
                                   scal + 3, s, &pb.bg));
  }
  SMFS_HIP(hipMemcpyAsync(stats, scal + 2, 8 * 4, hipMemcpyDeviceToHost, s));
  SMFS_HIP(hipStreamSynchronize(s));
  return SMFS_OK;
}

void fill_out(Problem &pb, const SolveStats &ss, const double *post, int precision, smfs_out *out) {
  out->iterations = ss.iterations;
  out->true_checks = ss.true_checks;
  out->floor_iteration = ss.floor_it;
  out->floor_rel_residual = ss.floor_rel;
  out->refinements = ss.refinements;
  out->rel_residual = ss.rel_residual;
  out->true_rel_residual = ss.rhs_norm > 0 ? ss.res_norm / ss.rhs_norm : 0.0;
  out->lambda_inf = post[0];
  out->eps_res_max = (out->u_check && pb.C) ? post[1] : -1.0;
  out->abs_res_max = (out->u_check && pb.C && post[3] > 0) ? post[2] / post[3] : -1.0;
  const bool mixed = is_mixed(precision) && pb.n_free > 0 && pb.fac32_ready;
  out->pair_evals = (int64_t)(ss.applies + ss.applies64) * pb.pairs_per_apply +
                    ((out->u_check) ? pb.C * pb.S : 0);
  out->pair_evals_f32 = mixed ? (int64_t)ss.applies * pb.pairs_f32 : 0;
  if (precision == SMFS_MIXED_EQ && eq_enabled(pb)) {
    // exact FP64 pairs and FP32 equivalent-source pairs of the EQ products
    out->pair_evals = (int64_t)ss.applies64 * pb.pairs_per_apply + (int64_t)ss.applies * pb.pairs_eq_exact +
                      ((out->u_check) ? pb.C * pb.S : 0);
    out->pair_evals_f32 = (int64_t)ss.applies * pb.pairs_eq_far;
  }
}

}  // namespace smfs

extern "C" {

int smfs_solve_resistance(smfs_problem *pb, const double *rbm, smfs_out *out, smfs_stream stream) {
  SMFS_READY(pb);
  if (!rbm || !out) { set_error("smfs_solve_resistance: null argument"); return SMFS_E_INVALID_ARG; }
  hipStream_t s = (hipStream_t)stream;
  using clk = std::chrono::steady_clock;
  auto ms = [](clk::time_point a, clk::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
  };
  const int64_t n = 3 * pb->T, ld = pb->kry_ld;
  double *b = pb->d_vec + 2 * ld;
  double *x = out->mu ? out->mu : pb->d_vec + 3 * ld;
  auto t0 = clk::now();
  SMFS_HIP(launch_rhs(pb->T, pb->d_tgt, pb->d_tsph, pb->d_sw, pb->d_meta, rbm, b, s, &pb->bg));
  SMFS_HIP(hipStreamSynchronize(s));
  auto t1 = clk::now();
  const int precision = pb->prm.precision;
  Problem &P = *pb;
  Operator op = [&P, s](const double *v, double *y, int prec) { return apply(P, v, y, prec, s); };
  SolveStats ss;
  int rc = solve_system(*pb, n, op, b, x, precision, ss, s);
  if (rc) return rc;
  auto t2 = clk::now();
  double post[4] = {0, 0, 0, 0};
  rc = post_process(*pb, x, rbm, out, post, s);
  if (rc) return rc;
  auto t3 = clk::now();
  fill_out(*pb, ss, post, precision, out);
  out->t_rhs_ms = ms(t0, t1);
  out->t_gmres_ms = ms(t1, t2);
  out->t_post_ms = ms(t2, t3);
  return solve_status(ss);
}

int smfs_solve_mobility(smfs_problem *pb, const double *ft, smfs_out *out, smfs_stream stream) {
  SMFS_READY(pb);
  if (!ft || !out) { set_error("smfs_solve_mobility: null argument"); return SMFS_E_INVALID_ARG; }
  hipStream_t s = (hipStream_t)stream;
  using clk = std::chrono::steady_clock;
  auto ms = [](clk::time_point a, clk::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
  };
  const int64_t n3 = 3 * pb->T, n = n3 + 6 * (int64_t)pb->P, ld = pb->kry_ld;
  double *b = pb->d_vec + 2 * ld;
  double *x = pb->d_vec + 3 * ld;
  auto t0 = clk::now();
  const double sF = 1.0 / (6.0 * kPi * pb->prm.mu * pb->a),
               sT = 1.0 / (8.0 * kPi * pb->prm.mu * pb->a * pb->a * pb->a);
  // velocity rows: the spheres' own motion is unknown, so only -W u_inf
  // (zero in a quiescent fluid)
  SMFS_HIP(launch_rhs(pb->T, pb->d_tgt, pb->d_tsph, pb->d_sw, pb->d_meta, nullptr, b, s, &pb->bg));
  SMFS_HIP(launch_scale_ft(pb->P, ft, sF, sT, b + n3, s));
  SMFS_HIP(hipStreamSynchronize(s));
  auto t1 = clk::now();
  const int precision = pb->prm.precision;
  Problem &P = *pb;
  Operator op = [&P, s](const double *v, double *y, int prec) { return apply_mobility(P, v, y, prec, s); };
  SolveStats ss;
  int rc = solve_system(*pb, n, op, b, x, precision, ss, s);
  if (rc) return rc;
  auto t2 = clk::now();
  if (out->mu) SMFS_HIP(hipMemcpyAsync(out->mu, x, 8 * n3, hipMemcpyDeviceToDevice, s));
  if (out->rbm) SMFS_HIP(hipMemcpyAsync(out->rbm, x + n3, 8 * 6 * pb->P, hipMemcpyDeviceToDevice, s));
  double post[4] = {0, 0, 0, 0};
  rc = post_process(*pb, x, x + n3, out, post, s);
  if (rc) return rc;
  auto t3 = clk::now();
  fill_out(*pb, ss, post, precision, out);
  out->t_rhs_ms = ms(t0, t1);
  out->t_gmres_ms = ms(t1, t2);
  out->t_post_ms = ms(t2, t3);
  return solve_status(ss);
}

}  // extern "C"
