// Internal structures of libsmfs (host side plus the device tables).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/smfs.h"

namespace smfs {

void set_error(const std::string &msg);

#define SMFS_HIP(call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) {                                                         \
      ::smfs::set_error(std::string("HIP error ") + hipGetErrorString(e_) + " at " + \
                        __FILE__ + ":" + std::to_string(__LINE__));                 \
      return SMFS_E_DEVICE;                                                         \
    }                                                                               \
  } while (0)

// One directed near contact of a sphere.
struct Contact {
  int32_t other;
  double gap;      // surface gap in radii
  double axis[3];  // unit vector towards the neighbour
  int32_t n_im;    // image nodes on this contact's line
};

// Packing blocks of the source array: proxy Stokeslets, image Stokeslets,
// rotlets, potential dipoles (each sphere-major).
constexpr int kBlocks = 4;

// Background flow u_inf(x) = U + L x (eq. bc), L row-major: L[3i + j] =
// d u_inf_i / d x_j.  Passed by value to the kernels; on == 0: quiescent.
struct BgFlow {
  double U[3];
  double L[9];
  int32_t on;
};

// Per-sphere table entry read by the kernels.
struct SphereMeta {
  int64_t t0;             // first collocation node
  int32_t M;              // collocation nodes
  int32_t N;              // vector sources (all kinds)
  int64_t k0[kBlocks];    // first source of the sphere in each block (packed index)
  int32_t kn[kBlocks];    // sources of the sphere in each block
  int32_t fid;            // factor id
  int32_t rank;           // kept singular values of that factor
  int64_t s0;             // offset of this sphere's U^T mu entries in the s buffer
  double c[3];            // centre
};

// A contiguous run of packed sources inside one block.
struct SrcRange {
  int32_t begin, end, block, pad;
};

// Per-factor storage inside the workspace (element offsets of doubles).
struct FactorSlot {
  int32_t rows, cols;   // 3 M, 3 N'
  int32_t rank;
  int32_t rep;          // representative sphere
  int64_t u_off;        // U: rows x cols column-major (first rank columns used)
  int64_t vt_off;       // V stored row-major: cols rows of stride cols
  int64_t sig_off;      // sigma (cols)
};

// Work item of the batched row-dot kernels: one output row.
struct RowTask {
  int32_t sphere;
  int32_t row;
};

struct Problem {
  smfs_params prm;
  int32_t P = 0;
  double a = 1.0;
  std::vector<double> centers;             // P x 3
  std::vector<std::vector<Contact>> contacts;
  int32_t n_contacts = 0;
  bool small_gap = false;

  // node sets (host)
  std::vector<double> tgt;                 // T x 3
  std::vector<double> tw;                  // T (area weight)
  std::vector<int32_t> tsph;               // T
  std::vector<int64_t> toff;               // P + 1
  std::vector<double> src;                 // S x 3, packed by kind
  std::vector<int32_t> skind, ssph;        // S
  std::vector<int64_t> koff[kBlocks];      // per block: P + 1 global offsets
  std::vector<double> chk;                 // C x 3
  std::vector<int32_t> csph;               // C
  int64_t T = 0, S = 0, C = 0;
  int64_t nk[3] = {0, 0, 0};               // per kind (S = proxy + image blocks)
  int64_t nb[kBlocks] = {0, 0, 0, 0};      // per block

  // factors
  std::vector<int32_t> fid_of;             // P
  std::vector<FactorSlot> factors;
  bool factors_ready = false;

  // workspace
  char *ws = nullptr;
  size_t ws_bytes = 0;
  bool bound = false;
  size_t need_bytes = 0, factor_bytes = 0;
  // device arrays (pointers into the workspace)
  double *d_tgt = nullptr, *d_sw = nullptr, *d_src = nullptr, *d_lamhat = nullptr;
  double *d_chk = nullptr, *d_fac = nullptr, *d_part = nullptr, *d_s = nullptr;
  int32_t *d_tsph = nullptr, *d_csph = nullptr;
  int4 *d_tiles = nullptr, *d_eval_tiles = nullptr;
  int4 *d_stiles = nullptr;                // one-sphere tiles (SMFS_MIXED far field, block sums, near sums)
  // mixed precision arrays
  float *d_tgt32 = nullptr, *d_src32 = nullptr, *d_str32 = nullptr, *d_part32 = nullptr;
  float *d_s32 = nullptr, *d_fac32 = nullptr;
  int32_t *d_free = nullptr;
  double *d_centers = nullptr;             // P x 3
  SrcRange *d_ranges = nullptr;            // [plain ranges | mixed FP64 ranges]
  int32_t n_free = 0, n_splits32 = 1;
  int32_t n_rng_plain = 0, n_rng_mixed = 0;
  int64_t rng_total_plain = 0, rng_total_mixed = 0;
  int64_t n_utask_c = 0, n_vtask_c = 0;    // tasks of contact spheres (a prefix)
  bool fac32_ready = false;
  SphereMeta *d_meta = nullptr;
  FactorSlot *d_fslots = nullptr;
  RowTask *d_utask = nullptr, *d_vtask = nullptr;
  int32_t *d_vmap = nullptr;               // packed source index of local source j, per sphere
  int4 *d_btask_u = nullptr, *d_btask_v = nullptr;  // block apply: (sphere, first row)
  int64_t n_btask_u = 0, n_btask_v = 0;
  int64_t cols_total = 0;                  // sum of factor columns over spheres
  bool skip_shared = false;                // setup leaves factor 0 (imported) alone
  int32_t svd_sweeps = 0;                  // Jacobi sweeps of the last set-up (largest over calls)
  BgFlow bg{};                             // background flow of the boundary data (off: quiescent)
  // equivalent-source far field (SMFS_MIXED_EQ)
  int32_t n_eq = 0;                        // equivalent points per sphere (0: off)
  std::vector<int32_t> near_off, near_idx; // per sphere: near contact-free spheres (free indices)
  double *d_eqE = nullptr;                 // 3 n_eq x 3 n_proxy, column-major
  float *d_eqq32 = nullptr;                // n_free x 3 n_eq equivalent strengths
  float *d_eqpt32 = nullptr;               // n_eq x 3 points relative to a centre
  int32_t *d_near_off = nullptr, *d_near_idx = nullptr;
  int32_t n_splits_eq = 0;
  bool eq_ready = false;
  int64_t pairs_eq_far = 0, pairs_eq_exact = 0;
  double *d_kry = nullptr, *d_vec = nullptr, *d_red = nullptr;
  int64_t n_tiles = 0, n_utask = 0, n_vtask = 0, n_vmap = 0;
  int64_t n_stiles = 0;
  int32_t n_splits = 1;
  int32_t n_splits_chk = 1;
  int64_t kry_ld = 0;
  int64_t part_cap = 0;                    // doubles in d_part
  int64_t red_cap = 0;                     // doubles in d_red
  int32_t kry_vecs = 0;

  // host mirrors of tables
  std::vector<SphereMeta> meta;
  std::vector<int4> tiles, stiles;
  std::vector<int32_t> vmap_off;           // P + 1 (offsets into d_vmap)

  void *rocblas = nullptr;                 // rocblas_handle for setup
  int64_t pairs_per_apply = 0;
  int64_t pairs_kind[3] = {0, 0, 0};       // per product, by source kind
  int64_t pairs_f32 = 0;                   // mixed precision: pairs with contact-free sources

  // per-launch event timing (smfs_profile)
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<size_t, size_t>> ev_direct, ev_pinv, ev_mixed64, ev_far32;
  std::vector<std::pair<size_t, size_t>> ev_bdirect, ev_bpinv;
  std::vector<std::pair<size_t, size_t>> ev_eqfar, ev_eqnear, ev_eqq;
  int32_t prof_nrhs = 0;                   // right-hand sides of the profiled block products
};

// geometry.cpp
int build_geometry(Problem &pb);
void spiral_points(int n, double r, std::vector<double> &out);
void build_near_lists(Problem &pb, double sep);
// tables.cpp
void build_tiles(const Problem &pb, std::vector<int4> &tiles, int tile_targets);
size_t workspace_layout(Problem &pb, bool assign);
int upload_tables(Problem &pb, hipStream_t s);
int rank_tables(Problem &pb, hipStream_t s);
// api.hip
int transform(Problem &pb, const double *mu, double *lam, hipStream_t s);
int record_event(Problem &pb, hipStream_t s, size_t &idx);
int32_t direct_splits(int64_t n_tiles, int64_t S);
bool valid_precision(int p);
bool is_mixed(int p);
bool eq_enabled(const Problem &pb);
// svd.hip: the device Jacobi SVD (QR, one-sided Jacobi on R, U = Q U_R)
struct JacPlan {
  int w = 8, rows = 4, npad = 0, nbk = 0, npairs = 0;
  bool wave = false;   // pair tasks of one wave (blocks of at most 768 columns)
  size_t work = 0;
  size_t a = 0, tau = 0, t = 0, tau2 = 0, x = 0, v = 0, wbuf = 0, off = 0, sig = 0, fro = 0, perm = 0, rank = 0, ptrs = 0, sched = 0, skip = 0;
  size_t total = 0;
};
}  // namespace smfs
typedef struct _rocblas_handle *rocblas_handle;
namespace smfs {
int jacobi_plan(rocblas_handle h, int m, int n, int nb, JacPlan &p);
int jacobi_svd_batch(rocblas_handle h, const JacPlan &p, char *scratch, int m, int n, int nb,
                     double *const *U, double *const *Vs, double *const *Ss, double trunc, int *ranks,
                     int *sweeps_out, hipStream_t s);
// block.hip
size_t block_apply_bytes(const Problem &pb, int32_t nrhs);
int block_apply_on(Problem &pb, int32_t nrhs, const double *mu, double *y, int64_t ld, char *base,
                   hipStream_t s);

}  // namespace smfs

struct smfs_problem : smfs::Problem {};

#define SMFS_READY(pb)                                                        \
  do {                                                                        \
    if (!(pb) || !(pb)->bound) { ::smfs::set_error("problem not bound"); return SMFS_E_STATE; } \
    if (!(pb)->factors_ready) { ::smfs::set_error("factors not set up"); return SMFS_E_STATE; } \
  } while (0)
