// Many right-hand sides: block product with G_hat and lock-step GMRES.
//
// The preconditioned operator (Section 2.2, eq. resistance) is the same for
// every right-hand side, so nrhs systems share one pass over the geometry:
// the direct sum computes each pair's separation and 1/|r| once per run of
// kBlockRun vectors, and the per-sphere pseudo-inverse (eq. transform)
// becomes two small GEMMs per sphere on FP64 MFMA.  Each system keeps its
// own Krylov basis, Hessenberg matrix and Givens rotations; the Arnoldi
// steps of all systems run together in batched kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/smfs.h"
#include "internal.h"
#include "kernels.h"

namespace smfs {
namespace {

constexpr double kPiB = 3.14159265358979323846;
constexpr size_t kAlignB = 256;

size_t up(size_t v) { return (v + kAlignB - 1) / kAlignB * kAlignB; }

// Regions of a caller-provided block workspace.
struct BlockLayout {
  double *lamb = nullptr;   // S x nrhs x 3 strengths (source-major)
  double *sblk = nullptr;   // nrhs x lds: Sigma^-1 U^T mu per sphere
  double *part = nullptr;   // [split][nrhs][3T] partial sums (one more slice: near proxies)
  float *str32 = nullptr;   // mixed: FP32 proxy strengths [proxy][nrhs][3]
  float *part32 = nullptr;  // mixed: FP32 partial sums [split32][nrhs][3T]
  float *q32b = nullptr;    // SMFS_MIXED_EQ: equivalent strengths [free][n_eq][nrhs][3]
  double *kry = nullptr;    // (m + 1) x nrhs x ld Krylov vectors
  double *vec = nullptr;    // 4 x nrhs x ld: w, r, b, x
  double *red = nullptr;    // reduction partials and small per-system arrays
  int64_t lds = 0, ld = 0;
  int32_t nsplit = 1, m = 0, nch = 1, ldh = 0;
  int32_t nsplit32 = 0;     // FP32 far-field splits (0: no contact-free sphere)
  int32_t nsplit_eq = 0;    // equivalent-source splits (0: form off)
  size_t bytes = 0;
};

BlockLayout block_layout(const Problem &pb, int32_t nrhs, int32_t m, char *base) {
  BlockLayout L;
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off = up(off + b);
    return o;
  };
  const int64_t n = 3 * pb.T;
  L.ld = (n + 31) / 32 * 32;
  L.lds = (pb.cols_total + 31) / 32 * 32;
  L.m = m;
  const int64_t nz = (nrhs + kBlockRun - 1) / kBlockRun;
  L.nsplit = direct_splits(pb.n_stiles * nz, pb.S);
  L.nch = mdot_chunks(n);
  L.ldh = m + 2;
  // the last run of right-hand sides reads (and ignores) up to kBlockRun - 1
  // strengths past the end of the block
  const size_t o_lamb = take(sizeof(double) * (3 * pb.S * nrhs + 3 * kBlockRun));
  const size_t o_s = take(sizeof(double) * L.lds * nrhs);
  const bool eq = eq_enabled(pb);
  const size_t o_part = take(sizeof(double) * (L.nsplit + (eq ? 1 : 0)) * nrhs * n);
  // mixed precision: FP32 strengths of the proxies (the last run reads up to
  // kBlockRun - 1 past the end) and FP32 partial sums of the far field
  if (pb.n_free > 0)
    L.nsplit32 = std::min<int32_t>(direct_splits(pb.n_stiles * nz, (int64_t)pb.n_free * pb.prm.n_proxy),
                                   std::max(1, pb.n_free));
  if (eq)
    L.nsplit_eq = std::min<int32_t>(direct_splits(pb.n_stiles * nz, (int64_t)pb.n_free * pb.n_eq),
                                    std::max(1, pb.n_free));
  const size_t o_str32 = take(sizeof(float) * (3 * pb.nb[0] * nrhs + 3 * kBlockRun));
  const size_t o_part32 =
      take(sizeof(float) * std::max<int64_t>(1, (int64_t)std::max(L.nsplit32, L.nsplit_eq) * nrhs * n));
  // the last run of right-hand sides reads up to kBlockRun - 1 past the end
  const size_t o_q32b = take(sizeof(float) * (eq ? (size_t)3 * pb.n_free * pb.n_eq * nrhs + 3 * kBlockRun : 1));
  size_t o_kry = 0, o_vec = 0, o_red = 0;
  if (m > 0) {
    o_kry = take(sizeof(double) * (size_t)(m + 1) * nrhs * L.ld);
    o_vec = take(sizeof(double) * 4 * (size_t)nrhs * L.ld);
    o_red = take(sizeof(double) * ((size_t)nrhs * (m + 1) * L.nch + 4 * (size_t)nrhs * L.ldh + 64));
  }
  L.bytes = off;
  if (base) {
    L.lamb = (double *)(base + o_lamb);
    L.sblk = (double *)(base + o_s);
    L.part = (double *)(base + o_part);
    L.str32 = (float *)(base + o_str32);
    L.part32 = (float *)(base + o_part32);
    L.q32b = (float *)(base + o_q32b);
    if (m > 0) {
      L.kry = (double *)(base + o_kry);
      L.vec = (double *)(base + o_vec);
      L.red = (double *)(base + o_red);
    }
  }
  return L;
}

int check_ws(const Problem &pb, int32_t nrhs, int32_t m, void *ws, size_t ws_bytes, BlockLayout &L) {
  if (nrhs <= 0 || nrhs > 65535) { set_error("nrhs must be in [1, 65535]"); return SMFS_E_INVALID_ARG; }
  if (!ws || ((uintptr_t)ws % kAlignB) != 0) {
    set_error("block workspace must be a 256-byte aligned device pointer");
    return SMFS_E_INVALID_ARG;
  }
  L = block_layout(pb, nrhs, m, (char *)ws);
  if (ws_bytes < L.bytes) { set_error("block workspace too small"); return SMFS_E_NOMEM; }
  return SMFS_OK;
}

// Y = G_hat M for the nrhs vectors of stride ld.  Mixed precision
// (SMFS_MIXED_FAR, or SMFS_MIXED: the block pseudo-inverse is FP64 in both):
// the proxies of contact-free spheres are summed in FP32 from FP32 copies of
// their FP64 strengths, every other pair in FP64.

int apply_block(Problem &pb, const BlockLayout &L, int32_t nrhs, const double *mu, double *y,
                int64_t ld, hipStream_t s, int precision = SMFS_FP64) {
  if (precision == SMFS_MIXED_EQ && !eq_enabled(pb)) precision = SMFS_FP64;   // nothing to approximate
  if (precision == SMFS_MIXED_EQ && !pb.eq_ready) {
    set_error("SMFS_MIXED_EQ block product before smfs_setup_far_field");
    return SMFS_E_STATE;
  }
  const bool eqf = precision == SMFS_MIXED_EQ;
  const bool mixed = is_mixed(precision) && L.nsplit32 > 0;
  size_t e0 = 0, e1 = 0, e2 = 0;
  int rc;
  if (pb.prof && (rc = record_event(pb, s, e0))) return rc;
  SMFS_HIP(launch_pinv_block(pb.d_btask_u, pb.n_btask_u, pb.d_btask_v, pb.n_btask_v, pb.d_meta,
                             pb.d_fslots, pb.d_fac, mu, ld, nrhs, L.sblk, L.lds, L.lamb,
                             2.0 * pb.prm.mu, s));
  if (pb.prof && (rc = record_event(pb, s, e1))) return rc;
  BlockDirectArgs a;
  a.tiles = pb.d_stiles;
  a.n_tiles = pb.n_stiles;
  a.tgt = pb.d_tgt;
  a.T = pb.T;
  a.src = pb.d_src;
  a.lamb = L.lamb;
  a.nrhs = nrhs;
  a.meta = pb.d_meta;
  a.ranges = mixed ? pb.d_ranges + pb.n_rng_plain : pb.d_ranges;
  a.n_ranges = mixed ? pb.n_rng_mixed : pb.n_rng_plain;
  a.range_total = mixed ? pb.rng_total_mixed : pb.rng_total_plain;
  a.n_splits = L.nsplit;
  a.part = L.part;
  SMFS_HIP(launch_direct_block(a, s));
  int32_t ns64 = L.nsplit, ns32 = mixed ? L.nsplit32 : 0;
  if (eqf) {
    // the contact spheres' sources are in the FP64 sum above; the near
    // contact-free proxies into one more FP64 slice, every other
    // contact-free sphere through its equivalent sources
    EqArgs f;
    f.tiles = pb.d_tiles;
    f.n_tiles = pb.n_tiles;
    f.tsph = pb.d_tsph;
    f.tgt = pb.d_tgt;
    f.eqpt32 = pb.d_eqpt32;
    f.q32 = nullptr;
    f.centers = pb.d_centers;
    f.free_ids = pb.d_free;
    f.near_off = pb.d_near_off;
    f.near_idx = pb.d_near_idx;
    f.n_free = pb.n_free;
    f.n_eq = pb.n_eq;
    f.n_splits = L.nsplit_eq;
    f.T = pb.T;
    f.part32 = L.part32;
    SMFS_HIP(launch_eq_block(a, f, pb.d_eqE, pb.prm.n_proxy, L.q32b, L.part + (int64_t)L.nsplit * nrhs * 3 * pb.T,
                             L.part32, s));
    ns64 = L.nsplit + 1;
    ns32 = L.nsplit_eq;
  } else if (mixed) {
    SMFS_HIP(launch_to_f32(3 * pb.nb[0] * nrhs, L.lamb, L.str32, s));
    Far32Args f = far32_args(pb);
    f.n_splits = L.nsplit32;
    SMFS_HIP(launch_far_block_f32(f, L.str32, nrhs, L.part32, s));
  }
  if (pb.prof) {
    if ((rc = record_event(pb, s, e2))) return rc;
    pb.ev_bpinv.emplace_back(e0, e1);
    pb.ev_bdirect.emplace_back(e1, e2);
    pb.prof_nrhs = nrhs;
  }
  SMFS_HIP(launch_reduce_block(3 * pb.T, nrhs, ns64, L.part, ns32, L.part32, mu, ld, pb.d_sw,
                               1.0 / (8.0 * kPiB * pb.prm.mu), y, ld, s));
  return SMFS_OK;
}

struct BlockStats {
  std::vector<int32_t> its;
  std::vector<double> est;      // GMRES residual estimate per system
  std::vector<char> conv;
  int32_t steps = 0;            // block products in the Krylov iterations
  int32_t refinements = 0;      // mixed: restarts from FP64 residuals after the estimates met tol
};

// Pinned host buffer released on scope exit.
struct Pinned {
  double *p = nullptr;
  ~Pinned() {
    if (p) (void)hipHostFree(p);
  }
};

// Lock-step GMRES(m) on G_hat x_q = b_q, x_q(0) = 0, for q < nrhs.  B and X
// are blocks of stride L.ld.  Classical Gram-Schmidt applied twice, as in
// the single-vector solver; a converged system is frozen (its restart
// vector is zero, so its later Arnoldi columns are zero and ignored).
int gmres_block(Problem &pb, const BlockLayout &L, int32_t nrhs, const double *B, double *X,
                double tol, int max_it, BlockStats &st, hipStream_t s, int precision = SMFS_FP64) {
  // mixed products inside the cycles; every restart takes the FP64 true
  // residual, and a mixed solve whose systems all stand converged while
  // some FP64 residual misses restarts from it up to twice (systems above
  // the tolerance go on)
  const bool mixed = is_mixed(precision) && L.nsplit32 > 0;
  int refinements = 0;
  const int64_t n = 3 * pb.T, ld = L.ld;
  const int m = L.m, ldh = L.ldh, nch = L.nch;
  const int64_t blk = (int64_t)nrhs * ld;   // one Krylov "column" of all systems
  double *V = L.kry;
  double *W = L.vec, *R = L.vec + blk;
  double *part = L.red;
  double *h = part + (int64_t)nrhs * (m + 1) * nch;
  double *h2 = h + (int64_t)nrhs * ldh;
  double *cf = h2 + (int64_t)nrhs * ldh;
  double *beta = cf + (int64_t)nrhs * ldh;   // nrhs x ldh (first entry used)
  Pinned hp;
  const size_t hp_n = 3 * (size_t)nrhs * ldh;
  SMFS_HIP(hipHostMalloc((void **)&hp.p, sizeof(double) * hp_n, hipHostMallocDefault));
  double *hh = hp.p, *hh2 = hp.p + (size_t)nrhs * ldh, *hb = hp.p + 2 * (size_t)nrhs * ldh;

  st.its.assign(nrhs, 0);
  st.est.assign(nrhs, 0.0);
  st.conv.assign(nrhs, 0);
  st.steps = 0;
  SMFS_HIP(launch_fill(blk, 0.0, X, s));
  SMFS_HIP(launch_norm_scale_block(const_cast<double *>(B), ld, nrhs, n, part, nch, beta, ldh, false, s));
  SMFS_HIP(hipMemcpyAsync(hb, beta, sizeof(double) * nrhs * ldh, hipMemcpyDeviceToHost, s));
  SMFS_HIP(hipStreamSynchronize(s));
  std::vector<double> bnorm(nrhs), g((size_t)nrhs * (m + 1)), cs((size_t)nrhs * m), sn((size_t)nrhs * m);
  std::vector<double> H((size_t)nrhs * (m + 1) * m), y(m), cfh((size_t)nrhs * ldh);
  std::vector<int> jdone(nrhs, 0);
  std::vector<char> active(nrhs, 0);
  for (int q = 0; q < nrhs; ++q) {
    bnorm[q] = hb[(size_t)q * ldh];
    if (bnorm[q] == 0.0) st.conv[q] = 1;
  }
  SMFS_HIP(hipMemcpyAsync(R, B, sizeof(double) * blk, hipMemcpyDeviceToDevice, s));
  std::vector<double> rn(bnorm);   // residual norms at the start of a cycle
  int total = 0;
  while (true) {
    // V_0 = R / beta for active systems, 0 for frozen ones
    int n_act = 0;
    for (int q = 0; q < nrhs; ++q) {
      active[q] = !st.conv[q] && rn[q] > 0.0;
      hb[(size_t)q * ldh] = active[q] ? rn[q] : 0.0;
      n_act += active[q];
      jdone[q] = 0;
    }
    if (n_act == 0) break;
    SMFS_HIP(hipMemcpyAsync(V, R, sizeof(double) * blk, hipMemcpyDeviceToDevice, s));
    SMFS_HIP(hipMemcpyAsync(beta, hb, sizeof(double) * nrhs * ldh, hipMemcpyHostToDevice, s));
    SMFS_HIP(launch_scale_block(V, ld, nrhs, n, beta, ldh, s));
    std::fill(g.begin(), g.end(), 0.0);
    for (int q = 0; q < nrhs; ++q) g[(size_t)q * (m + 1)] = active[q] ? rn[q] : 0.0;
    std::vector<char> running(active);
    for (int j = 0; j < m; ++j) {
      double *vj = V + (int64_t)j * blk, *vj1 = V + (int64_t)(j + 1) * blk;
      int rc = apply_block(pb, L, nrhs, vj, vj1, ld, s, precision);
      if (rc) return rc;
      ++st.steps;
      SMFS_HIP(launch_arnoldi_block(V, ld, nrhs, j + 1, vj1, n, part, nch, h, ldh, s));
      SMFS_HIP(launch_arnoldi_block(V, ld, nrhs, j + 1, vj1, n, part, nch, h2, ldh, s));
      SMFS_HIP(launch_norm_scale_block(vj1, ld, nrhs, n, part, nch, h + (j + 1), ldh, true, s));
      SMFS_HIP(hipMemcpyAsync(hh, h, sizeof(double) * nrhs * ldh, hipMemcpyDeviceToHost, s));
      SMFS_HIP(hipMemcpyAsync(hh2, h2, sizeof(double) * nrhs * ldh, hipMemcpyDeviceToHost, s));
      SMFS_HIP(hipStreamSynchronize(s));
      ++total;
      int n_run = 0;
      for (int q = 0; q < nrhs; ++q) {
        if (!running[q]) continue;
        double *Hq = &H[(size_t)q * (m + 1) * m];
        double *col = Hq + (size_t)j * (m + 1);
        const double *a = hh + (size_t)q * ldh, *a2 = hh2 + (size_t)q * ldh;
        for (int i = 0; i <= j + 1; ++i) col[i] = a[i] + (i <= j ? a2[i] : 0.0);
        double *c = &cs[(size_t)q * m], *sv = &sn[(size_t)q * m], *gq = &g[(size_t)q * (m + 1)];
        for (int i = 0; i < j; ++i) {
          const double t = c[i] * col[i] + sv[i] * col[i + 1];
          col[i + 1] = -sv[i] * col[i] + c[i] * col[i + 1];
          col[i] = t;
        }
        const double den = std::hypot(col[j], col[j + 1]);
        c[j] = den > 0 ? col[j] / den : 1.0;
        sv[j] = den > 0 ? col[j + 1] / den : 0.0;
        col[j] = den;
        col[j + 1] = 0.0;
        gq[j + 1] = -sv[j] * gq[j];
        gq[j] = c[j] * gq[j];
        jdone[q] = j + 1;
        st.its[q] += 1;
        st.est[q] = std::fabs(gq[j + 1]) / bnorm[q];
        if (st.est[q] <= tol) {
          st.conv[q] = 1;
          running[q] = 0;
        } else if (a[j + 1] == 0.0 || total >= max_it) {
          running[q] = 0;
        }
        n_run += running[q];
      }
      if (n_run == 0) break;
    }
    // y_q = H_q^-1 g_q, x_q += V_q y_q
    std::fill(cfh.begin(), cfh.end(), 0.0);
    int nv = 0;
    for (int q = 0; q < nrhs; ++q) {
      const int jd = jdone[q];
      nv = std::max(nv, jd);
      const double *Hq = &H[(size_t)q * (m + 1) * m];
      const double *gq = &g[(size_t)q * (m + 1)];
      for (int i = jd - 1; i >= 0; --i) {
        double t = gq[i];
        for (int c = i + 1; c < jd; ++c) t -= Hq[(size_t)c * (m + 1) + i] * y[c];
        y[i] = t / Hq[(size_t)i * (m + 1) + i];
      }
      for (int i = 0; i < jd; ++i) cfh[(size_t)q * ldh + i] = y[i];
    }
    SMFS_HIP(hipMemcpyAsync(cf, cfh.data(), sizeof(double) * nrhs * ldh, hipMemcpyHostToDevice, s));
    SMFS_HIP(launch_combine_block(V, ld, nrhs, nv, cf, ldh, X, ld, n, s));
    SMFS_HIP(hipStreamSynchronize(s));
    bool more = false;
    for (int q = 0; q < nrhs; ++q) more = more || (!st.conv[q]);
    const bool refine = mixed && !more && refinements < 2;
    if ((!more && !refine) || total >= max_it) break;
    if (refine) ++refinements;
    // restart from the true residuals
    int rc = apply_block(pb, L, nrhs, X, W, ld, s);
    if (rc) return rc;
    ++st.steps;
    SMFS_HIP(launch_sub(blk, B, W, R, s));
    SMFS_HIP(launch_norm_scale_block(R, ld, nrhs, n, part, nch, beta, ldh, false, s));
    SMFS_HIP(hipMemcpyAsync(hb, beta, sizeof(double) * nrhs * ldh, hipMemcpyDeviceToHost, s));
    SMFS_HIP(hipStreamSynchronize(s));
    bool all_conv = true, any_miss = false;
    for (int q = 0; q < nrhs; ++q) {
      rn[q] = hb[(size_t)q * ldh];
      if (bnorm[q] == 0.0) continue;
      const bool met = rn[q] / bnorm[q] <= tol;
      if (refine) st.conv[q] = met ? 1 : 0;       // checked against the FP64 residual
      if (met && !st.conv[q]) st.conv[q] = 1;
      if (met) st.est[q] = rn[q] / bnorm[q];
      all_conv = all_conv && st.conv[q];
      any_miss = any_miss || !met;
    }
    // The last running systems met the tolerance on this FP64 residual
    // while others stand converged on their mixed estimates alone: this
    // restart becomes their refinement, as if the estimates had met first.
    if (mixed && !refine && all_conv && any_miss && refinements < 2) {
      ++refinements;
      for (int q = 0; q < nrhs; ++q)
        if (bnorm[q] != 0.0) st.conv[q] = rn[q] / bnorm[q] <= tol ? 1 : 0;
    }
    st.refinements = refinements;
  }
  return SMFS_OK;
}

}  // namespace

// Block product on a workspace at base (at least block_apply_bytes bytes,
// 256-byte aligned), for other entry points of the library.
size_t block_apply_bytes(const Problem &pb, int32_t nrhs) { return block_layout(pb, nrhs, 0, nullptr).bytes; }

int block_apply_on(Problem &pb, int32_t nrhs, const double *mu, double *y, int64_t ld, char *base,
                   hipStream_t s) {
  const BlockLayout L = block_layout(pb, nrhs, 0, base);
  return apply_block(pb, L, nrhs, mu, y, ld, s, SMFS_FP64);
}

}  // namespace smfs

using namespace smfs;

extern "C" {

int smfs_block_workspace_bytes(const smfs_problem *pb, int32_t nrhs, int32_t restart, size_t *bytes) {
  if (!pb || !bytes || nrhs <= 0 || nrhs > 65535 || restart < 0 || restart > 20000) {
    set_error("smfs_block_workspace_bytes: bad argument");
    return SMFS_E_INVALID_ARG;
  }
  if (!pb->bound) { set_error("problem not bound"); return SMFS_E_STATE; }
  *bytes = block_layout(*pb, nrhs, restart, nullptr).bytes;
  return SMFS_OK;
}

int smfs_apply_block(smfs_problem *pb, int32_t nrhs, const double *mu, double *y, int64_t ld,
                     int32_t precision, void *ws, size_t ws_bytes, smfs_stream stream) {
  SMFS_READY(pb);
  if (!mu || !y || ld < 3 * pb->T) { set_error("smfs_apply_block: bad vectors"); return SMFS_E_INVALID_ARG; }
  if (!valid_precision(precision)) { set_error("smfs_apply_block: bad precision"); return SMFS_E_INVALID_ARG; }
  BlockLayout L;
  int rc = check_ws(*pb, nrhs, 0, ws, ws_bytes, L);
  if (rc) return rc;
  const char *a0 = (const char *)mu, *a1 = a0 + 8 * (nrhs * ld);
  const char *b0 = (const char *)y, *b1 = b0 + 8 * (nrhs * ld);
  if (a0 < b1 && b0 < a1) { set_error("smfs_apply_block: mu and y overlap"); return SMFS_E_INVALID_ARG; }
  return apply_block(*pb, L, nrhs, mu, y, ld, (hipStream_t)stream, precision);
}

int smfs_solve_resistance_block(smfs_problem *pb, int32_t nrhs, const double *rbm, int32_t restart,
                                void *ws, size_t ws_bytes, smfs_block_out *out, smfs_stream stream) {
  SMFS_READY(pb);
  if (!rbm || !out || restart <= 0 || restart > 20000) {
    set_error("smfs_solve_resistance_block: bad argument");
    return SMFS_E_INVALID_ARG;
  }
  BlockLayout L;
  int rc = check_ws(*pb, nrhs, restart, ws, ws_bytes, L);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  using clk = std::chrono::steady_clock;
  auto ms = [](clk::time_point a, clk::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
  };
  const int64_t n = 3 * pb->T, ld = L.ld, blk = (int64_t)nrhs * ld, P = pb->P;
  double *W = L.vec, *R = L.vec + blk, *B = L.vec + 2 * blk, *X = L.vec + 3 * blk;
  auto t0 = clk::now();
  SMFS_HIP(launch_fill(blk, 0.0, B, s));
  for (int q = 0; q < nrhs; ++q)
    SMFS_HIP(launch_rhs(pb->T, pb->d_tgt, pb->d_tsph, pb->d_sw, pb->d_meta, rbm + 6 * P * q,
                        B + (int64_t)q * ld, s, &pb->bg));
  BlockStats st;
  rc = gmres_block(*pb, L, nrhs, B, X, pb->prm.gmres_tol, pb->prm.gmres_max_it, st, s, pb->prm.precision);
  if (rc) return rc;
  // true residuals in FP64
  rc = apply_block(*pb, L, nrhs, X, W, ld, s);
  if (rc) return rc;
  SMFS_HIP(launch_sub(blk, B, W, R, s));
  double *red = L.red + (int64_t)nrhs * (L.m + 1) * L.nch;
  double *rn = red, *bn = red + nrhs;
  SMFS_HIP(launch_norm_scale_block(R, ld, nrhs, n, L.red, L.nch, rn, 1, false, s));
  SMFS_HIP(launch_norm_scale_block(B, ld, nrhs, n, L.red, L.nch, bn, 1, false, s));
  std::vector<double> norms(2 * (size_t)nrhs);
  SMFS_HIP(hipMemcpyAsync(norms.data(), red, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, s));
  SMFS_HIP(hipStreamSynchronize(s));
  auto t1 = clk::now();
  // strengths, forces and torques per system (single-vector kernels)
  for (int q = 0; q < nrhs; ++q) {
    const double *xq = X + (int64_t)q * ld;
    if (out->ft) {
      rc = transform(*pb, xq, pb->d_lamhat, s);
      if (rc) return rc;
      SMFS_HIP(launch_force_torque(pb->P, pb->d_meta, pb->d_src, pb->d_lamhat, out->ft + 6 * P * q, s));
    }
    if (out->mu) SMFS_HIP(hipMemcpyAsync(out->mu + n * q, xq, 8 * n, hipMemcpyDeviceToDevice, s));
  }
  SMFS_HIP(hipStreamSynchronize(s));
  auto t2 = clk::now();
  int nconv = 0, maxit = 0, ntrue = 0;
  for (int q = 0; q < nrhs; ++q) {
    nconv += st.conv[q] ? 1 : 0;
    maxit = std::max(maxit, st.its[q]);
    if (out->iterations) out->iterations[q] = st.its[q];
    const double tr = norms[nrhs + q] > 0 ? norms[q] / norms[nrhs + q] : 0.0;
    if (out->true_rel_residual) out->true_rel_residual[q] = tr;
    ntrue += tr <= pb->prm.gmres_tol ? 1 : 0;
  }
  out->refinements = st.refinements;
  if (is_mixed(pb->prm.precision))
    out->pair_evals_f32 = (int64_t)st.steps * nrhs * pb->pairs_f32;
  out->max_iterations = maxit;
  out->n_converged = nconv;
  out->t_gmres_ms = ms(t0, t1);
  out->t_post_ms = ms(t1, t2);
  out->pair_evals = (int64_t)(st.steps + 1) * nrhs * pb->pairs_per_apply;
  if (pb->prm.precision == SMFS_MIXED_EQ && eq_enabled(*pb)) {
    // exact and equivalent-source pairs of the EQ products, FP64 residuals
    out->pair_evals = (int64_t)st.steps * nrhs * pb->pairs_eq_exact + (int64_t)nrhs * pb->pairs_per_apply;
    out->pair_evals_f32 = (int64_t)st.steps * nrhs * pb->pairs_eq_far;
  }
  // OK only when every FP64 true residual met the tolerance
  if (ntrue == nrhs) return SMFS_OK;
  return nconv == nrhs ? SMFS_STAGNATED : SMFS_NOT_CONVERGED;
}

}  // extern "C"
