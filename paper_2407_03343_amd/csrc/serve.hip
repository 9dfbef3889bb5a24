// Serving: continuous batching of independent resistance solves.
//
// Each request is a full problem of its own (geometry, factors, Krylov
// basis) living in a slice of one device arena.  Set-up worker threads
// admit requests in arrival order when their slice fits and a slot is free,
// and build them, each on its own stream (tables, the per-contact SVDs,
// right-hand side, first Krylov vector), while the resident requests keep
// iterating on the main stream.  Several workers overlap the host-side
// latency of the small SVDs with one another.
//
// smfs_server_step advances every resident request by one GMRES iteration
// with one launch per kernel for all of them (launch_serve_product,
// launch_serve_arnoldi), reads the new Hessenberg columns back in one copy
// and applies each request's Givens rotations on the host, exactly as the
// single-problem solver does.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/smfs.h"
#include "internal.h"
#include "kernels.h"

namespace smfs {

DirectArgs direct_args(Problem &pb, const double *str, bool mixed);
int setup_factors(Problem &pb, char *scratch, size_t scratch_bytes, hipStream_t s);
int apply(Problem &pb, const double *mu, double *y, int precision, hipStream_t s);

namespace {

constexpr size_t kAl = 256;
constexpr double kPiS = 3.14159265358979323846;

size_t al(size_t v) { return (v + kAl - 1) / kAl * kAl; }

double clock_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator of 256-byte aligned slices of the arena, with
// coalescing of neighbouring free slices.
class Arena {
 public:
  void init(size_t cap) {
    free_.clear();
    free_[0] = cap;
    used_ = peak_ = 0;
  }
  bool fits(size_t bytes) const {
    bytes = al(bytes);
    for (auto &f : free_)
      if (f.second >= bytes) return true;
    return false;
  }
  bool take(size_t bytes, size_t &off) {
    bytes = al(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      off = it->first;
      const size_t rest = it->second - bytes, o2 = it->first + bytes;
      free_.erase(it);
      if (rest) free_[o2] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }
  void give(size_t off, size_t bytes) {
    bytes = al(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t peak() const { return peak_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0, peak_ = 0;
};

enum class St { kQueued, kSetup, kReady, kRunning, kDone };

struct Req {
  int64_t id = 0;
  smfs_problem *pb = nullptr;
  int32_t P = 0;
  std::vector<double> rbm;
  St state = St::kQueued;
  int status = SMFS_OK;
  std::string err;
  size_t off = 0, bytes = 0;
  bool has_mem = false;
  // GMRES state (one restart cycle)
  int m = 0, j = 0, total = 0, restarts = 0, refinements = 0;
  bool converged = false;
  double bnorm = 0.0, est = 0.0;
  std::vector<double> H, cs, sn, g;
  // results
  std::vector<double> ft;
  double true_rel = 0.0;
  int64_t pair_evals_f32 = 0;
  double t_arrival = 0, t_admit = 0, t_start = 0, t_done = 0;
  int64_t pair_evals = 0;
};

}  // namespace
}  // namespace smfs

using namespace smfs;

namespace smfs {
namespace {
// A set-up worker: its own thread, stream, rocBLAS handle and SVD scratch
// (a slice of the caller's memory: rocSOLVER's work arrays, then the
// batched SVD inputs and outputs).
struct Worker {
  hipStream_t s = nullptr;
  rocblas_handle rb = nullptr;
  void *work = nullptr;              // rocSOLVER's work arrays (the handle's user workspace)
  size_t work_bytes = 0;
  void *scratch = nullptr;           // batched SVD inputs, outputs, status words
  size_t scratch_bytes = 0;
  std::map<std::pair<int, int>, int> cap;   // SVD batch count per block shape
  std::thread th;
};
constexpr size_t kSvdScratch = (size_t)4 << 30;   // default per worker
constexpr size_t kSvdBatch = 256;    // most blocks per batched SVD call (fixed per shape)
}  // namespace
}  // namespace smfs

struct smfs_server {
  smfs_params prm{};
  double radius = 1.0;
  int device = 0;
  int32_t max_queued = 0;        // 0: no limit
  char *arena = nullptr;         // part of the caller's memory
  size_t arena_bytes = 0;
  Arena alloc;
  int32_t max_active = 1;
  hipStream_t s_main = nullptr;
  std::vector<Worker> workers;
  double *f0 = nullptr;          // shared contact-free factor (U, V^T, sigma)
  int64_t f0_elems = 0;
  int32_t f0_rank = 0, f0_rows = 0, f0_cols = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Req *> queue;
  std::vector<Req *> ready, active;
  int32_t in_setup = 0;
  int32_t max_batch = 64;        // requests set up together
  std::unordered_map<int64_t, Req *> reqs;
  int64_t next_id = 1;
  bool stop = false;
  ServeDesc *d_desc = nullptr, *h_desc = nullptr;
  double *d_tick = nullptr;      // Gram-Schmidt coefficients of the slots (device only)
  int32_t ldt = 0;               // doubles per request in the tick buffer
  // GMRES cycle state of the slots on the device, and its host mirror
  ServeGivens *d_gv = nullptr, *h_gv = nullptr;
  double *d_gst = nullptr, *h_gst = nullptr;  // H, cs, sn, g of each slot
  int64_t gstride = 0;           // doubles per slot in d_gst
  int32_t iters_per_step = 8;    // GMRES iterations per smfs_server_step
  smfs_server_stats st{};
};

namespace {

void free_request_memory(smfs_server *srv, Req *r) {
  // caller holds srv->mu
  if (r->has_mem) {
    srv->alloc.give(r->off, r->bytes);
    r->has_mem = false;
  }
}

void drop_problem(Req *r) {
  if (r->pb) {
    r->pb->rocblas = nullptr;   // the server's handle
    smfs_problem_destroy(r->pb);
    r->pb = nullptr;
  }
}

// Tables and the shared factor of request r in its arena slice.
int bind_request(smfs_server *srv, Worker &wk, Req *r) {
  Problem &pb = *r->pb;
  int rc = smfs_bind(r->pb, srv->arena + r->off, r->bytes, wk.s);
  if (rc) return rc;
  if (pb.factors[0].rep >= 0) {
    const FactorSlot &f = pb.factors[0];
    if (f.rows != srv->f0_rows || f.cols != srv->f0_cols) {
      set_error("serving: shared factor shape differs from the server's");
      return SMFS_E_STATE;
    }
    SMFS_HIP(hipMemcpyAsync(pb.d_fac + f.u_off, srv->f0, sizeof(double) * srv->f0_elems,
                            hipMemcpyDeviceToDevice, wk.s));
    pb.factors[0].rank = srv->f0_rank;
  }
  return SMFS_OK;
}

// Right-hand side, x = 0 and V_0 = b / ||b|| of a request whose factors are set.
int prepare_request(Worker &wk, Req *r) {
  Problem &pb = *r->pb;
  hipStream_t s = wk.s;
  int rc = rank_tables(pb, s);
  if (rc) return rc;
  if (!pb.factors_ready) { set_error("serving: a factor has rank 0"); return SMFS_E_SVD; }
  const int64_t ld = pb.kry_ld, n = 3 * pb.T;
  double *b = pb.d_vec + 2 * ld, *x = pb.d_vec + 3 * ld, *rb = pb.d_vec + 5 * ld;
  double *scal = pb.d_red + pb.red_cap - 8;
  const int32_t nch = mdot_chunks(n);
  SMFS_HIP(hipMemcpyAsync(rb, r->rbm.data(), sizeof(double) * 6 * r->P, hipMemcpyHostToDevice, s));
  SMFS_HIP(launch_rhs(pb.T, pb.d_tgt, pb.d_tsph, pb.d_sw, pb.d_meta, rb, b, s));
  SMFS_HIP(launch_fill(n, 0.0, x, s));
  SMFS_HIP(hipMemcpyAsync(pb.d_kry, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  SMFS_HIP(launch_norm_scale(pb.d_kry, n, pb.d_red, nch, scal, scal + 1, s));
  double bn = 0.0;
  SMFS_HIP(hipMemcpyAsync(&bn, scal, sizeof(double), hipMemcpyDeviceToHost, s));
  SMFS_HIP(hipStreamSynchronize(s));
  r->bnorm = bn;
  r->m = pb.kry_vecs - 1;
  r->H.assign((size_t)(r->m + 1) * r->m, 0.0);
  r->cs.assign(r->m, 0.0);
  r->sn.assign(r->m, 0.0);
  r->g.assign(r->m + 1, 0.0);
  r->g[0] = bn;
  r->j = 0;
  return SMFS_OK;
}

// The self-block factorisations (Section 2.2, eq. transform) of every contact sphere of a
// batch of requests, grouped by block shape across requests: batched SVDs
// per shape, because a batched SVD of small blocks costs little more than a
// single one.  Every call has the same batch count for a given shape (the
// last chunk is padded with copies of its first block), so that a block's
// factors do not depend on which other blocks share the call: a request's
// result is then the same alone and in any mix.  Results are written into
// the requests' factor slots; a request whose SVD fails gets its status.
void factor_batch(Worker &wk, std::vector<Req *> &batch) {
  struct Job {
    Req *r;
    int fid;
  };
  std::map<std::pair<int, int>, std::vector<Job>> groups;
  for (Req *r : batch) {
    Problem &pb = *r->pb;
    for (size_t f = 1; f < pb.factors.size(); ++f)
      if (pb.factors[f].rep >= 0) groups[{pb.factors[f].rows, pb.factors[f].cols}].push_back(Job{r, (int)f});
  }
  hipStream_t s = wk.s;
  auto fail = [](Req *r, int rc) {
    if (r->status == SMFS_OK) {
      r->status = rc;
      r->err = smfs_last_error();
    }
  };
  for (auto &grp : groups) {
    const int m = grp.first.first, n = grp.first.second;
    const size_t per = (size_t)m * n;
    const size_t slot = ((size_t)m * n + (size_t)n * n + n + 31) / 32 * 32;
    const size_t each = 8 * (per + slot + n) + 4 + 3 * kAl;
    size_t cap = 0;
    {
      // blocks per call for this shape: as many as the scratch holds (at most
      // kSvdBatch) whose SVD work arrays also fit the worker's workspace; it
      // depends on the shape and the worker's memory only, so every call of
      // a shape has the same batch count
      auto it = wk.cap.find({m, n});
      if (it != wk.cap.end()) {
        cap = (size_t)it->second;
      } else {
        cap = std::max<size_t>(1, std::min<size_t>(kSvdBatch, wk.scratch_bytes / each));
        double *fake = reinterpret_cast<double *>((uintptr_t)4096);
        rocblas_int *ifake = reinterpret_cast<rocblas_int *>((uintptr_t)4096);
        while (true) {
          size_t need = 0;
          rocblas_start_device_memory_size_query(wk.rb);
          const rocblas_status q = rocsolver_dgesvd_strided_batched(
              wk.rb, rocblas_svect_singular, rocblas_svect_singular, m, n, fake, m, (rocblas_stride)per,
              fake, (rocblas_stride)slot, fake, m, (rocblas_stride)slot, fake, n, (rocblas_stride)slot,
              fake, n, rocblas_outofplace, ifake, (rocblas_int)cap);
          rocblas_stop_device_memory_size_query(wk.rb, &need);
          const bool ok = q == rocblas_status_success || q == rocblas_status_size_increased ||
                          q == rocblas_status_size_unchanged;
          if ((ok && need <= wk.work_bytes) || cap == 1) break;
          cap = std::max<size_t>(1, cap / 2);
        }
        wk.cap[{m, n}] = (int)cap;
      }
    }
    std::vector<Job> &jobs = grp.second;
    for (size_t j0 = 0; j0 < jobs.size(); j0 += cap) {
      const int nb = (int)std::min(cap, jobs.size() - j0);   // real blocks in this call
      const int nc = (int)cap;                                // blocks in the call
      char *base = (char *)wk.scratch;
      double *A = (double *)base;
      double *Out = (double *)(base + al(8 * per * nc));
      double *E = (double *)((char *)Out + al(8 * slot * nc));
      rocblas_int *info = (rocblas_int *)((char *)E + al(8 * (size_t)n * nc));
      int rc = SMFS_OK;
      for (int q = 0; q < nb && !rc; ++q) {
        const Job &jb = jobs[j0 + q];
        Problem &pb = *jb.r->pb;
        const FactorSlot &fs = pb.factors[jb.fid];
        const SphereMeta &mk = pb.meta[fs.rep];
        if (launch_assemble_block(pb.d_tgt, pb.d_sw, pb.d_src, pb.d_meta, fs.rep, mk.M, mk.N, pb.prm.mu,
                                  A + (size_t)q * per, s) != hipSuccess) {
          set_error("serving: block assembly failed");
          rc = SMFS_E_DEVICE;
        }
      }
      for (int q = nb; q < nc && !rc; ++q)
        if (hipMemcpyAsync(A + (size_t)q * per, A, 8 * per, hipMemcpyDeviceToDevice, s) != hipSuccess) {
          set_error("serving: block padding failed");
          rc = SMFS_E_DEVICE;
        }
      std::vector<rocblas_int> hinfo(nb, 0);
      std::vector<double> sv((size_t)nb * n, 0.0);
      if (!rc) {
        const rocblas_status st = rocsolver_dgesvd_strided_batched(
            wk.rb, rocblas_svect_singular, rocblas_svect_singular, m, n, A, m, (rocblas_stride)per,
            Out + per + (size_t)n * n, (rocblas_stride)slot, Out, m, (rocblas_stride)slot, Out + per, n,
            (rocblas_stride)slot, E, n, rocblas_outofplace, info, nc);
        if (st != rocblas_status_success) {
          set_error("rocsolver_dgesvd_strided_batched failed with status " + std::to_string((int)st));
          rc = SMFS_E_SVD;
        }
      }
      if (!rc) {
        hipError_t e = hipMemcpyAsync(hinfo.data(), info, sizeof(rocblas_int) * nb, hipMemcpyDeviceToHost, s);
        for (int q = 0; q < nb && e == hipSuccess; ++q)
          e = hipMemcpyAsync(sv.data() + (size_t)q * n, Out + (size_t)q * slot + per + (size_t)n * n,
                             8 * (size_t)n, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
          set_error(std::string("serving: reading SVD results failed: ") + hipGetErrorString(e));
          rc = SMFS_E_DEVICE;
        }
      }
      for (int q = 0; q < nb; ++q) {
        const Job &jb = jobs[j0 + q];
        Problem &pb = *jb.r->pb;
        if (rc) { fail(jb.r, rc); continue; }
        const double *sq = sv.data() + (size_t)q * n;
        if (hinfo[q] != 0 || !(sq[0] > 0)) {
          set_error("SVD did not converge (info " + std::to_string(hinfo[q]) + ", sigma_1 " +
                    std::to_string(sq[0]) + ")");
          fail(jb.r, SMFS_E_SVD);
          continue;
        }
        int rank = 0;
        while (rank < n && sq[rank] > pb.prm.trunc_rel * sq[0]) ++rank;
        FactorSlot &fs = pb.factors[jb.fid];
        fs.rank = rank;
        if (hipMemcpyAsync(pb.d_fac + fs.u_off, Out + (size_t)q * slot,
                           8 * ((size_t)m * n + (size_t)n * n + n), hipMemcpyDeviceToDevice, s) != hipSuccess) {
          set_error("serving: factor copy failed");
          fail(jb.r, SMFS_E_DEVICE);
        }
      }
      // the scratch is reused by the next chunk
      if (hipStreamSynchronize(s) != hipSuccess) {
        set_error("serving: factor copy failed");
        for (int q = 0; q < nb; ++q) fail(jobs[j0 + q].r, SMFS_E_DEVICE);
      }
    }
  }
}

// factor_batch with the device Jacobi SVD (svd_method SMFS_SVD_JACOBI): per
// block shape, chunks of as many blocks as the worker's memory holds (its
// rocSOLVER part and its scratch, which are contiguous, serve as one region
// laid out by the Jacobi plan); U, V and sigma are written straight into
// the requests' factor slots.  A block's sweeps stop when its own rotations
// do, and the way its QR reflectors are applied depends on its shape only,
// so its factors do not depend on the other blocks of the call.
void factor_batch_jacobi(Worker &wk, std::vector<Req *> &batch) {
  struct Job {
    Req *r;
    int fid;
  };
  std::map<std::pair<int, int>, std::vector<Job>> groups;
  for (Req *r : batch) {
    Problem &pb = *r->pb;
    for (size_t f = 1; f < pb.factors.size(); ++f)
      if (pb.factors[f].rep >= 0) groups[{pb.factors[f].rows, pb.factors[f].cols}].push_back(Job{r, (int)f});
  }
  hipStream_t s = wk.s;
  char *region = (char *)wk.work;
  const size_t region_bytes = wk.work_bytes + wk.scratch_bytes;
  auto fail = [](Req *r, int rc) {
    if (r->status == SMFS_OK) {
      r->status = rc;
      r->err = smfs_last_error();
    }
  };
  for (auto &grp : groups) {
    const int m = grp.first.first, n = grp.first.second;
    std::vector<Job> &jobs = grp.second;
    int cap = (int)std::min<size_t>(kSvdBatch, jobs.size());
    int prc = SMFS_OK;
    while (true) {
      JacPlan jp;
      prc = jacobi_plan(wk.rb, m, n, cap, jp);
      if (prc != SMFS_OK) break;   // the shape itself is refused (its error is set)
      if (jp.total <= region_bytes) break;
      if (cap == 1) { cap = 0; break; }
      cap = std::max(1, cap / 2);
    }
    if (prc != SMFS_OK) {
      for (const Job &jb : jobs) fail(jb.r, prc);
      continue;
    }
    if (cap == 0) {
      set_error("serving: a " + std::to_string(m) + " x " + std::to_string(n) +
                " block does not fit the set-up worker's memory for the device SVD");
      for (const Job &jb : jobs) fail(jb.r, SMFS_E_NOMEM);
      continue;
    }
    for (size_t j0 = 0; j0 < jobs.size(); j0 += cap) {
      const int nb = (int)std::min<size_t>(cap, jobs.size() - j0);
      JacPlan jp;
      int rc = jacobi_plan(wk.rb, m, n, nb, jp);
      double *A = (double *)(region + jp.work);
      std::vector<double *> U(nb), V(nb), S(nb);
      for (int q = 0; q < nb && !rc; ++q) {
        const Job &jb = jobs[j0 + q];
        Problem &pb = *jb.r->pb;
        const FactorSlot &fs = pb.factors[jb.fid];
        const SphereMeta &mk = pb.meta[fs.rep];
        if (launch_assemble_block(pb.d_tgt, pb.d_sw, pb.d_src, pb.d_meta, fs.rep, mk.M, mk.N, pb.prm.mu,
                                  A + (size_t)q * m * n, s) != hipSuccess) {
          set_error("serving: block assembly failed");
          rc = SMFS_E_DEVICE;
        }
        U[q] = pb.d_fac + fs.u_off;
        V[q] = pb.d_fac + fs.vt_off;
        S[q] = pb.d_fac + fs.sig_off;
      }
      std::vector<int> ranks(nb, 0);
      int sweeps = 0;
      if (!rc) rc = jacobi_svd_batch(wk.rb, jp, region, m, n, nb, U.data(), V.data(), S.data(),
                                     jobs[j0].r->pb->prm.trunc_rel, ranks.data(), &sweeps, s);
      // the region's rocSOLVER part is the handle's workspace again
      if (rocblas_set_workspace(wk.rb, wk.work, wk.work_bytes) != rocblas_status_success && !rc) {
        set_error("rocblas_set_workspace failed");
        rc = SMFS_E_DEVICE;
      }
      for (int q = 0; q < nb; ++q) {
        const Job &jb = jobs[j0 + q];
        if (rc) { fail(jb.r, rc); continue; }
        Problem &pb = *jb.r->pb;
        pb.factors[jb.fid].rank = ranks[q];
        pb.svd_sweeps = std::max(pb.svd_sweeps, sweeps);
      }
    }
  }
}

void worker_main(smfs_server *srv, int wi) {
  (void)hipSetDevice(srv->device);
  Worker &wk = srv->workers[wi];
  while (true) {
    std::vector<Req *> batch;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      auto admissible = [srv] {
        if (srv->queue.empty()) return false;
        const int32_t resident = (int32_t)(srv->active.size() + srv->ready.size()) + srv->in_setup;
        return resident < srv->max_active && srv->alloc.fits(srv->queue.front()->bytes);
      };
      srv->cv.wait(lk, [&] { return srv->stop || admissible(); });
      if (srv->stop) return;
      // every request that can be admitted now, in arrival order
      while (admissible() && (int32_t)batch.size() < srv->max_batch) {
        Req *r = srv->queue.front();
        srv->queue.pop_front();
        srv->alloc.take(r->bytes, r->off);
        r->has_mem = true;
        r->state = St::kSetup;
        r->t_admit = clock_s();
        ++srv->in_setup;
        batch.push_back(r);
      }
    }
    const double t0 = clock_s();
    std::vector<Req *> ok;
    for (Req *r : batch) {
      const int rc = bind_request(srv, wk, r);
      if (rc) {
        r->status = rc;
        r->err = smfs_last_error();
      } else {
        ok.push_back(r);
      }
    }
    if (srv->prm.svd_method == SMFS_SVD_JACOBI) factor_batch_jacobi(wk, ok);
    else factor_batch(wk, ok);
    for (Req *r : ok)
      if (r->status == SMFS_OK) {
        const int rc = prepare_request(wk, r);
        if (rc) {
          r->status = rc;
          r->err = smfs_last_error();
        }
      }
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->in_setup -= (int32_t)batch.size();
    srv->st.setup_ms += (clock_s() - t0) * 1e3;
    ++srv->st.setup_batches;
    bool freed = false;
    for (Req *r : batch) {
      if (r->status != SMFS_OK) {
        r->state = St::kDone;
        r->t_done = clock_s();
        free_request_memory(srv, r);
        drop_problem(r);
        ++srv->st.failed;
        freed = true;
      } else {
        r->state = St::kReady;
        srv->ready.push_back(r);
      }
    }
    if (freed) srv->cv.notify_all();
  }
}

// True residual, strengths, forces and torques; results to the host.
int complete_request(smfs_server *srv, Req *r) {
  Problem &pb = *r->pb;
  hipStream_t s = srv->s_main;
  const int64_t ld = pb.kry_ld, n = 3 * pb.T;
  double *w = pb.d_vec, *rv = pb.d_vec + ld, *b = pb.d_vec + 2 * ld, *x = pb.d_vec + 3 * ld;
  double *ftd = pb.d_vec + 4 * ld;
  double *scal = pb.d_red + pb.red_cap - 8;
  const int32_t nch = mdot_chunks(n);
  int rc = apply(pb, x, w, SMFS_FP64, s);
  if (rc) return rc;
  SMFS_HIP(launch_sub(n, b, w, rv, s));
  SMFS_HIP(launch_norm2(rv, n, pb.d_red, nch, scal, s));
  rc = transform(pb, x, pb.d_lamhat, s);
  if (rc) return rc;
  SMFS_HIP(launch_force_torque(pb.P, pb.d_meta, pb.d_src, pb.d_lamhat, ftd, s));
  r->ft.assign(6 * (size_t)r->P, 0.0);
  double rn = 0.0;
  SMFS_HIP(hipMemcpyAsync(r->ft.data(), ftd, sizeof(double) * 6 * r->P, hipMemcpyDeviceToHost, s));
  SMFS_HIP(hipMemcpyAsync(&rn, scal, sizeof(double), hipMemcpyDeviceToHost, s));
  SMFS_HIP(hipStreamSynchronize(s));
  r->true_rel = r->bnorm > 0 ? rn / r->bnorm : 0.0;
  r->pair_evals = (int64_t)(r->total + r->restarts + 1) * pb.pairs_per_apply;
  if (is_mixed(srv->prm.precision) && pb.n_free > 0) r->pair_evals_f32 = (int64_t)r->total * pb.pairs_f32;
  return SMFS_OK;
}

// x += V y for the finished cycle of r; returns the cycle length used.
int combine_cycle(smfs_server *srv, Req *r) {
  Problem &pb = *r->pb;
  const int jd = r->j, m = r->m;
  if (jd == 0) return SMFS_OK;
  std::vector<double> y(jd);
  for (int i = jd - 1; i >= 0; --i) {
    double t = r->g[i];
    for (int c = i + 1; c < jd; ++c) t -= r->H[(size_t)c * (m + 1) + i] * y[c];
    y[i] = t / r->H[(size_t)i * (m + 1) + i];
  }
  const int64_t ld = pb.kry_ld, n = 3 * pb.T;
  const int32_t nch = mdot_chunks(n);
  double *cf = pb.d_red + (int64_t)nch * (m + 2) + 2 * (m + 2);
  SMFS_HIP(hipMemcpyAsync(cf, y.data(), sizeof(double) * jd, hipMemcpyHostToDevice, srv->s_main));
  SMFS_HIP(launch_combine(pb.d_kry, ld, jd, cf, pb.d_vec + 3 * ld, n, srv->s_main));
  SMFS_HIP(hipStreamSynchronize(srv->s_main));
  return SMFS_OK;
}

// Restart from the true residual; sets *done when it already meets the tolerance.
int restart_cycle(smfs_server *srv, Req *r, bool *done) {
  Problem &pb = *r->pb;
  hipStream_t s = srv->s_main;
  const int64_t ld = pb.kry_ld, n = 3 * pb.T;
  double *w = pb.d_vec, *rv = pb.d_vec + ld, *b = pb.d_vec + 2 * ld, *x = pb.d_vec + 3 * ld;
  double *scal = pb.d_red + pb.red_cap - 8;
  const int32_t nch = mdot_chunks(n);
  int rc = apply(pb, x, w, SMFS_FP64, s);
  if (rc) return rc;
  ++r->restarts;
  SMFS_HIP(launch_sub(n, b, w, rv, s));
  SMFS_HIP(hipMemcpyAsync(pb.d_kry, rv, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  SMFS_HIP(launch_norm_scale(pb.d_kry, n, pb.d_red, nch, scal, scal + 1, s));
  double beta = 0.0;
  SMFS_HIP(hipMemcpyAsync(&beta, scal, sizeof(double), hipMemcpyDeviceToHost, s));
  SMFS_HIP(hipStreamSynchronize(s));
  std::fill(r->H.begin(), r->H.end(), 0.0);
  std::fill(r->g.begin(), r->g.end(), 0.0);
  r->g[0] = beta;
  r->j = 0;
  if (beta / r->bnorm <= srv->prm.gmres_tol) {
    r->converged = true;
    r->est = beta / r->bnorm;
    *done = true;
  }
  return SMFS_OK;
}

}  // namespace

extern "C" {

double smfs_server_clock(void) { return clock_s(); }

int smfs_server_config_default(smfs_server_config *c) {
  if (!c) { set_error("null config"); return SMFS_E_INVALID_ARG; }
  std::memset(c, 0, sizeof(*c));
  c->radius = 1.0;
  c->max_active = 64;
  c->setup_workers = 1;
  c->max_queued = 0;
  c->precision = SMFS_FP64;
  c->worker_scratch_bytes = kSvdScratch;
  c->iters_per_step = 8;
  c->setup_batch = 64;
  return SMFS_OK;
}

}  // extern "C"

namespace smfs {
namespace {

// Fixed part of the server's device memory (before the arena): the shared
// factor, descriptors and Hessenberg readback of the slots, every worker's
// scratch.  Offsets from the start of the caller's memory.
struct ServerLayout {
  size_t f0 = 0, desc = 0, tick = 0, gv = 0, gst = 0, workers = 0, arena = 0;
  size_t worker_bytes = 0, work_bytes = 0;
  int64_t f0_elems = 0, gstride = 0;
  int32_t ldt = 0;
};

int server_layout(const smfs_params *p, const smfs_server_config *c, ServerLayout &L) {
  if (!p || !c || !(c->radius > 0) || c->max_active < 1 || c->max_active > 4096 || c->setup_workers < 1 ||
      c->setup_workers > 64 || c->max_queued < 0 || c->iters_per_step < 0 || c->iters_per_step > 1024 ||
      c->setup_batch < 0 || c->setup_batch > 64) {
    set_error("smfs_server: bad configuration");
    return SMFS_E_INVALID_ARG;
  }
  if (c->precision != SMFS_FP64 && c->precision != SMFS_MIXED_FAR) {
    set_error("smfs_server: serving runs SMFS_FP64 or SMFS_MIXED_FAR products");
    return SMFS_E_UNSUPPORTED;
  }
  // the shared factor's shape from a one-sphere problem (host geometry only)
  const double c0[3] = {0.0, 0.0, 0.0};
  double radius = c->radius;
  smfs_problem *t = nullptr;
  int rc = smfs_problem_create(p, 1, c0, &radius, &t);
  if (rc < 0) return rc;
  const FactorSlot &f = t->factors[0];
  L.f0_elems = (int64_t)f.rows * f.cols + (int64_t)f.cols * f.cols + f.cols;
  smfs_problem_destroy(t);
  const int64_t m = std::max(1, p->gmres_restart);
  L.ldt = 2 * ((int32_t)m + 2);
  L.gstride = ((m + 1) * m + 2 * m + (m + 1) + 31) / 32 * 32;
  L.worker_bytes = al(c->worker_scratch_bytes ? c->worker_scratch_bytes : kSvdScratch);
  // a quarter of each worker's scratch (at least 64 MiB) for rocSOLVER's work arrays
  L.work_bytes = al(std::max<size_t>((size_t)64 << 20, L.worker_bytes / 4));
  if (L.work_bytes >= L.worker_bytes) {
    set_error("smfs_server: worker scratch too small (at least 128 MiB)");
    return SMFS_E_INVALID_ARG;
  }
  size_t off = 0;
  L.f0 = off;
  off = al(off + sizeof(double) * (size_t)L.f0_elems);
  L.desc = off;
  off = al(off + sizeof(ServeDesc) * (size_t)c->max_active);
  L.tick = off;
  off = al(off + sizeof(double) * (size_t)L.ldt * c->max_active);
  L.gv = off;
  off = al(off + sizeof(ServeGivens) * (size_t)c->max_active);
  L.gst = off;
  off = al(off + sizeof(double) * (size_t)L.gstride * c->max_active);
  L.workers = off;
  off += L.worker_bytes * (size_t)c->setup_workers;
  L.arena = off;
  return SMFS_OK;
}

}  // namespace
}  // namespace smfs

extern "C" {

int smfs_server_memory_bytes(const smfs_params *p, const smfs_server_config *c, size_t *fixed_bytes) {
  if (!fixed_bytes) { set_error("null argument"); return SMFS_E_INVALID_ARG; }
  ServerLayout L;
  int rc = server_layout(p, c, L);
  if (rc) return rc;
  *fixed_bytes = L.arena;
  return SMFS_OK;
}

int smfs_server_create(const smfs_params *p, const smfs_server_config *c, void *dev_mem, size_t dev_bytes,
                       smfs_server **out) {
  if (!out || !dev_mem || ((uintptr_t)dev_mem) % kAl) {
    set_error("smfs_server_create: null argument or device memory not 256-byte aligned");
    return SMFS_E_INVALID_ARG;
  }
  *out = nullptr;
  ServerLayout L;
  int rc = server_layout(p, c, L);
  if (rc) return rc;
  if (dev_bytes <= L.arena) {
    set_error("smfs_server_create: " + std::to_string(dev_bytes) + " bytes of device memory leave no arena (" +
              std::to_string(L.arena) + " needed before it)");
    return SMFS_E_NOMEM;
  }
  smfs_server *srv = new smfs_server();
  srv->prm = *p;
  srv->prm.precision = c->precision;
  srv->radius = c->radius;
  srv->max_active = c->max_active;
  srv->max_queued = c->max_queued;
  char *base = (char *)dev_mem;
  srv->arena = base + L.arena;
  srv->arena_bytes = dev_bytes - L.arena;
  struct Guard {
    smfs_server *s;
    ~Guard() { if (s) smfs_server_destroy(s); }
  } guard{srv};
  SMFS_HIP(hipGetDevice(&srv->device));
  srv->alloc.init(srv->arena_bytes);
  SMFS_HIP(hipStreamCreate(&srv->s_main));
  srv->workers.resize(c->setup_workers);
  for (size_t i = 0; i < srv->workers.size(); ++i) {
    Worker &w = srv->workers[i];
    SMFS_HIP(hipStreamCreate(&w.s));
    if (rocblas_create_handle(&w.rb) != rocblas_status_success) {
      set_error("rocblas_create_handle failed");
      return SMFS_E_DEVICE;
    }
    rocblas_set_stream(w.rb, w.s);
    char *wb = base + L.workers + i * L.worker_bytes;
    w.work = wb;
    w.work_bytes = L.work_bytes;
    w.scratch = wb + L.work_bytes;
    w.scratch_bytes = L.worker_bytes - L.work_bytes;
  }
  Worker &w0 = srv->workers[0];
  // the shared factor from a single contact-free sphere, set up in the (still
  // empty) arena with worker 0's scratch
  {
    const double c0[3] = {0.0, 0.0, 0.0};
    double radius = c->radius;
    smfs_problem *t = nullptr;
    rc = smfs_problem_create(&srv->prm, 1, c0, &radius, &t);
    if (rc < 0) return rc;
    struct Drop {
      smfs_problem *t;
      ~Drop() { if (t) { t->rocblas = nullptr; smfs_problem_destroy(t); } }
    } drop{t};
    if (t->need_bytes > srv->arena_bytes) {
      set_error("smfs_server_create: the arena does not hold a one-sphere request");
      return SMFS_E_NOMEM;
    }
    if ((rc = smfs_bind(t, srv->arena, t->need_bytes, w0.s))) return rc;
    t->rocblas = w0.rb;
    if ((rc = setup_factors(*t, (char *)w0.work, L.worker_bytes, w0.s))) return rc;
    const FactorSlot &f = t->factors[0];
    srv->f0_rows = f.rows;
    srv->f0_cols = f.cols;
    srv->f0_rank = f.rank;
    srv->f0_elems = L.f0_elems;
    srv->f0 = (double *)(base + L.f0);
    SMFS_HIP(hipMemcpyAsync(srv->f0, t->d_fac + f.u_off, sizeof(double) * srv->f0_elems,
                            hipMemcpyDeviceToDevice, w0.s));
    SMFS_HIP(hipStreamSynchronize(w0.s));
  }
  // from here on rocSOLVER works in each worker's own slice
  for (Worker &w : srv->workers)
    if (rocblas_set_workspace(w.rb, w.work, w.work_bytes) != rocblas_status_success) {
      set_error("rocblas_set_workspace failed");
      return SMFS_E_DEVICE;
    }
  srv->ldt = L.ldt;
  srv->d_desc = (ServeDesc *)(base + L.desc);
  SMFS_HIP(hipHostMalloc((void **)&srv->h_desc, sizeof(ServeDesc) * c->max_active, hipHostMallocDefault));
  srv->d_tick = (double *)(base + L.tick);
  srv->d_gv = (ServeGivens *)(base + L.gv);
  srv->d_gst = (double *)(base + L.gst);
  srv->gstride = L.gstride;
  srv->iters_per_step = c->iters_per_step > 0 ? c->iters_per_step : 8;
  srv->max_batch = c->setup_batch > 0 ? c->setup_batch : 64;
  SMFS_HIP(hipHostMalloc((void **)&srv->h_gv, sizeof(ServeGivens) * c->max_active, hipHostMallocDefault));
  SMFS_HIP(hipHostMalloc((void **)&srv->h_gst, sizeof(double) * srv->gstride * c->max_active,
                         hipHostMallocDefault));
  srv->st.arena_bytes = srv->arena_bytes;
  for (int i = 0; i < c->setup_workers; ++i) srv->workers[i].th = std::thread(worker_main, srv, i);
  guard.s = nullptr;
  *out = srv;
  return SMFS_OK;
}

void smfs_server_destroy(smfs_server *srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv.notify_all();
  for (Worker &w : srv->workers)
    if (w.th.joinable()) w.th.join();
  if (srv->s_main) (void)hipStreamSynchronize(srv->s_main);
  for (Worker &w : srv->workers)
    if (w.s) (void)hipStreamSynchronize(w.s);
  for (auto &kv : srv->reqs) {
    drop_problem(kv.second);
    delete kv.second;
  }
  // the device memory is the caller's; host buffers, streams and handles are ours
  if (srv->h_desc) (void)hipHostFree(srv->h_desc);
  if (srv->h_gv) (void)hipHostFree(srv->h_gv);
  if (srv->h_gst) (void)hipHostFree(srv->h_gst);
  for (Worker &w : srv->workers) {
    if (w.rb) rocblas_destroy_handle(w.rb);
    if (w.s) (void)hipStreamDestroy(w.s);
  }
  if (srv->s_main) (void)hipStreamDestroy(srv->s_main);
  delete srv;
}

int smfs_server_submit(smfs_server *srv, int32_t P, const double *centers, const double *rbm,
                       double t_arrival, int64_t *id) {
  if (!srv || !centers || !rbm || !id || P <= 0) {
    set_error("smfs_server_submit: bad argument");
    return SMFS_E_INVALID_ARG;
  }
  for (int i = 0; i < 6 * P; ++i)
    if (!std::isfinite(rbm[i])) {
      set_error("smfs_server_submit: non-finite rigid motion");
      return SMFS_E_INVALID_ARG;
    }
  if (srv->max_queued > 0) {
    std::lock_guard<std::mutex> lk(srv->mu);
    if ((int32_t)srv->queue.size() >= srv->max_queued) {
      set_error("smfs_server_submit: queue full");
      return SMFS_E_AGAIN;
    }
  }
  const double now = clock_s();
  std::vector<double> radii(P, srv->radius);
  smfs_problem *pb = nullptr;
  int rc = smfs_problem_create(&srv->prm, P, centers, radii.data(), &pb);
  if (rc < 0) return rc;
  if (pb->need_bytes > srv->arena_bytes) {
    smfs_problem_destroy(pb);
    set_error("smfs_server_submit: request larger than the arena");
    return SMFS_E_NOMEM;
  }
  Req *r = new Req();
  r->pb = pb;
  r->P = P;
  r->rbm.assign(rbm, rbm + 6 * P);
  r->bytes = pb->need_bytes;
  r->t_arrival = t_arrival >= 0 ? t_arrival : now;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    r->id = srv->next_id++;
    srv->reqs[r->id] = r;
    srv->queue.push_back(r);
  }
  srv->cv.notify_all();
  *id = r->id;
  return SMFS_OK;
}

int smfs_server_step(smfs_server *srv, int32_t *n_active, int32_t *n_waiting) {
  if (!srv) { set_error("null server"); return SMFS_E_INVALID_ARG; }
  const double t0 = clock_s();
  std::vector<Req *> act;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    for (Req *r : srv->ready) {
      r->state = St::kRunning;
      r->t_start = t0;
      srv->active.push_back(r);
    }
    srv->ready.clear();
    act = srv->active;
  }
  hipStream_t s = srv->s_main;
  std::vector<Req *> finished;
  // zero right-hand sides finish at once (x = 0)
  std::vector<Req *> run;
  for (Req *r : act) {
    if (r->bnorm == 0.0) {
      r->converged = true;
      finished.push_back(r);
    } else {
      run.push_back(r);
    }
  }
  const int32_t nprob = (int32_t)run.size();
  if (nprob > 0) {
    int64_t tiles = 0, ut = 0, vt = 0, max_n = 0, stiles = 0, max_str32 = 0;
    int32_t max_splits = 1, max_nch = 1, max_splits32 = 0, max_j = 0;
    const int mh = srv->ldt / 2;
    const int64_t gs = srv->gstride;
    for (int32_t i = 0; i < nprob; ++i) {
      Req *r = run[i];
      Problem &pb = *r->pb;
      ServeDesc &d = srv->h_desc[i];
      const bool mixed = is_mixed(srv->prm.precision) && pb.n_free > 0;
      d.da = direct_args(pb, pb.d_lamhat, mixed);
      d.tile0 = tiles;
      d.fa = Far32Args{};
      d.stile0 = stiles;
      d.str32 = pb.d_str32;
      d.n_str32 = 3 * pb.nb[0];
      if (mixed) {
        d.fa = far32_args(pb);
        stiles += pb.n_stiles;
        max_splits32 = std::max(max_splits32, pb.n_splits32);
        max_str32 = std::max(max_str32, d.n_str32);
      }
      d.utask = pb.d_utask;
      d.vtask = pb.d_vtask;
      d.n_utask = pb.n_utask;
      d.n_vtask = pb.n_vtask;
      d.utask0 = ut;
      d.vtask0 = vt;
      d.fs = pb.d_fslots;
      d.fac = pb.d_fac;
      d.sbuf = pb.d_s;
      d.lam = pb.d_lamhat;
      d.n = 3 * pb.T;
      d.ld = pb.kry_ld;
      d.V = pb.d_kry;
      d.sw = pb.d_sw;
      d.c0 = 1.0 / (8.0 * kPiS * pb.prm.mu);
      d.gv = srv->d_gv + i;
      d.nch = mdot_chunks(d.n);
      d.red = pb.d_red;
      d.h = srv->d_tick + (int64_t)i * srv->ldt;
      d.h2 = d.h + mh;
      // the cycle state of slot i: header and H, cs, sn, g
      ServeGivens &G = srv->h_gv[i];
      G.j = r->j;
      G.m = r->m;
      G.active = 1;
      G.total = r->total;
      G.max_it = srv->prm.gmres_max_it;
      G.breakdown = 0;
      G.bnorm = r->bnorm;
      G.tol = srv->prm.gmres_tol;
      G.est = r->est;
      G.H = srv->d_gst + (int64_t)i * gs;
      G.cs = G.H + (int64_t)(r->m + 1) * r->m;
      G.sn = G.cs + r->m;
      G.g = G.sn + r->m;
      double *hs = srv->h_gst + (int64_t)i * gs;
      std::copy(r->H.begin(), r->H.end(), hs);
      std::copy(r->cs.begin(), r->cs.end(), hs + (G.cs - G.H));
      std::copy(r->sn.begin(), r->sn.end(), hs + (G.sn - G.H));
      std::copy(r->g.begin(), r->g.end(), hs + (G.g - G.H));
      tiles += pb.n_tiles;
      ut += pb.n_utask;
      vt += pb.n_vtask;
      max_n = std::max(max_n, d.n);
      max_splits = std::max(max_splits, pb.n_splits);
      max_nch = std::max(max_nch, d.nch);
      max_j = std::max(max_j, r->j);
    }
    SMFS_HIP(hipMemcpyAsync(srv->d_desc, srv->h_desc, sizeof(ServeDesc) * nprob, hipMemcpyHostToDevice, s));
    SMFS_HIP(hipMemcpyAsync(srv->d_gv, srv->h_gv, sizeof(ServeGivens) * nprob, hipMemcpyHostToDevice, s));
    SMFS_HIP(hipMemcpyAsync(srv->d_gst, srv->h_gst, sizeof(double) * gs * nprob, hipMemcpyHostToDevice, s));
    // iters_per_step iterations of every request with no host round trip:
    // each launch skips the requests whose cycle state went inactive; the
    // Arnoldi grids cover the longest possible basis (j grows by one per
    // iteration and stays below the cycle length)
    const int m_all = run[0]->m;
    for (int it = 0; it < srv->iters_per_step; ++it) {
      const int32_t max_nv = std::min(max_j + it + 1, m_all);
      SMFS_HIP(launch_serve_product(srv->d_desc, nprob, tiles, ut, vt, max_splits, max_n, stiles, max_splits32,
                                    max_str32, s));
      SMFS_HIP(launch_serve_arnoldi(srv->d_desc, nprob, max_nv, max_nch, max_n, s));
      SMFS_HIP(launch_serve_givens(srv->d_desc, nprob, s));
    }
    SMFS_HIP(hipMemcpyAsync(srv->h_gv, srv->d_gv, sizeof(ServeGivens) * nprob, hipMemcpyDeviceToHost, s));
    SMFS_HIP(hipMemcpyAsync(srv->h_gst, srv->d_gst, sizeof(double) * gs * nprob, hipMemcpyDeviceToHost, s));
    SMFS_HIP(hipStreamSynchronize(s));
    srv->st.tick_ms += (clock_s() - t0) * 1e3;
    ++srv->st.steps;
    srv->st.iterations += srv->iters_per_step;
    const double tol = srv->prm.gmres_tol;
    for (int32_t i = 0; i < nprob; ++i) {
      Req *r = run[i];
      const ServeGivens &G = srv->h_gv[i];
      const double *hs = srv->h_gst + (int64_t)i * gs;
      const int m = r->m;
      srv->st.request_iterations += G.total - r->total;
      r->j = G.j;
      r->total = G.total;
      r->est = G.est;
      std::copy(hs, hs + r->H.size(), r->H.begin());
      std::copy(hs + (int64_t)(m + 1) * m, hs + (int64_t)(m + 1) * m + m, r->cs.begin());
      std::copy(hs + (int64_t)(m + 1) * m + m, hs + (int64_t)(m + 1) * m + 2 * m, r->sn.begin());
      std::copy(hs + (int64_t)(m + 1) * m + 2 * m, hs + (int64_t)(m + 1) * m + 3 * m + 1, r->g.begin());
      if (G.active) continue;   // still iterating: nothing for the host
      bool done = false, refine = false;
      if (r->est <= tol) {
        r->converged = true;
        done = true;
        // mixed products: restart from the FP64 true residual (at most two
        // refinements); the request goes on when that residual is above tol
        refine = is_mixed(srv->prm.precision) && r->refinements < 2 &&
                 r->total < srv->prm.gmres_max_it;
      } else if (r->total >= srv->prm.gmres_max_it || G.breakdown) {
        done = true;
      }
      if (done || r->j == m) {
        int rc = combine_cycle(srv, r);
        if (!rc && (!done || refine)) {
          bool met = false;
          rc = restart_cycle(srv, r, &met);
          if (refine) {
            ++r->refinements;
            done = met;
            r->converged = met;
          } else {
            done = met;
          }
        }
        if (rc) {
          r->status = rc;
          r->err = smfs_last_error();
          done = true;
        }
      }
      if (done) finished.push_back(r);
    }
  }
  for (Req *r : finished) {
    if (r->status == SMFS_OK) {
      const int rc = complete_request(srv, r);
      if (rc) {
        r->status = rc;
        r->err = smfs_last_error();
      } else if (r->true_rel > srv->prm.gmres_tol) {
        // honest status: OK only when the FP64 true residual meets the tolerance
        r->status = r->converged ? SMFS_STAGNATED : SMFS_NOT_CONVERGED;
      }
    }
    r->t_done = clock_s();
  }
  int32_t na = 0, nw = 0;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    for (Req *r : finished) {
      r->state = St::kDone;
      free_request_memory(srv, r);
      drop_problem(r);
      if (r->status >= 0) ++srv->st.completed;
      else ++srv->st.failed;
    }
    if (!finished.empty()) {
      std::vector<Req *> keep;
      for (Req *r : srv->active)
        if (r->state != St::kDone) keep.push_back(r);
      srv->active.swap(keep);
    }
    na = (int32_t)srv->active.size();
    nw = (int32_t)(srv->queue.size() + srv->ready.size()) + srv->in_setup;
    srv->st.peak_active = std::max(srv->st.peak_active, (int32_t)act.size());
    srv->st.arena_peak = srv->alloc.peak();
    srv->st.step_ms += (clock_s() - t0) * 1e3;
  }
  if (!finished.empty()) srv->cv.notify_all();
  if (n_active) *n_active = na;
  if (n_waiting) *n_waiting = nw;
  return SMFS_OK;
}

int smfs_server_poll(smfs_server *srv, int64_t id, smfs_request_result *res, double *ft) {
  if (!srv || !res) { set_error("smfs_server_poll: bad argument"); return SMFS_E_INVALID_ARG; }
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(id);
  if (it == srv->reqs.end()) { set_error("smfs_server_poll: unknown request"); return SMFS_E_INVALID_ARG; }
  const Req *r = it->second;
  if (r->state != St::kDone) return 1;
  res->status = r->status;
  res->P = r->P;
  res->iterations = r->total;
  res->restarts = r->restarts;
  res->rel_residual = r->est;
  res->true_rel_residual = r->true_rel;
  res->t_arrival = r->t_arrival;
  res->t_admitted = r->t_admit;
  res->t_started = r->t_start;
  res->t_done = r->t_done;
  res->pair_evals = r->pair_evals;
  res->pair_evals_f32 = r->pair_evals_f32;
  res->refinements = r->refinements;
  std::snprintf(res->error, sizeof(res->error), "%s", r->err.c_str());
  if (ft && !r->ft.empty()) std::memcpy(ft, r->ft.data(), sizeof(double) * r->ft.size());
  return SMFS_OK;
}

int smfs_server_release(smfs_server *srv, int64_t id) {
  if (!srv) { set_error("null server"); return SMFS_E_INVALID_ARG; }
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(id);
  if (it == srv->reqs.end()) { set_error("smfs_server_release: unknown request"); return SMFS_E_INVALID_ARG; }
  if (it->second->state != St::kDone) { set_error("smfs_server_release: request not finished"); return SMFS_E_STATE; }
  delete it->second;
  srv->reqs.erase(it);
  return SMFS_OK;
}

int smfs_server_stats_read(smfs_server *srv, smfs_server_stats *st) {
  if (!srv || !st) { set_error("null argument"); return SMFS_E_INVALID_ARG; }
  std::lock_guard<std::mutex> lk(srv->mu);
  *st = srv->st;
  return SMFS_OK;
}

}  // extern "C"
