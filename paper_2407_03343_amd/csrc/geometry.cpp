// Host geometry: proxy spheres, image lines, collocation caps, area weights
// and residual check points of the image-enhanced MFS discretisation.
//
//  - proxy Stokeslets on radius R_p a and base collocation nodes on radius a
//    (Section 2.1), placed on a Fibonacci spiral (spherical designs are not
//    used): cos(theta_j) = 1 - (2j - 1)/n, phi_j = 2 pi j / golden mod 2 pi;
//  - image nodes c + a t_j e on the line towards each neighbour closer than
//    image_gap_cutoff, t_j from eq. (tj) with R_acc(delta) of eq. (Racc);
//  - two Fibonacci caps per contact around e with half-angles beta_1,2 and
//    alpha_i 3 n_im nodes each (eq. colloc_nbr), using
//    cos(theta_j) = 1 - j (1 - cos beta) / M_cap (the printed eq. thetacap
//    does not give caps of half-angle beta);
//  - weight of a node = area of its set / node count (Remark left-precond).
#include <algorithm>
#include <cmath>
#include <string>

#include "internal.h"

namespace smfs {

namespace {

constexpr double kPi = 3.14159265358979323846;

inline double golden() { return 0.5 * (1.0 + std::sqrt(5.0)); }

// Unit vector of spiral node j (1-based) of an n-node sphere set.
inline void spiral(int j, int n, double jshift, double out[3]) {
  double ct = 1.0 - (2.0 * j - 1.0) / n;
  double st = std::sqrt(std::fmax(0.0, 1.0 - ct * ct));
  double ph = std::fmod(2.0 * kPi * (j + jshift) / golden(), 2.0 * kPi);
  out[0] = st * std::cos(ph);
  out[1] = st * std::sin(ph);
  out[2] = ct;
}

inline void cross(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

inline double norm3(const double v[3]) { return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

// Frame (e1, e2) orthogonal to the contact axis e; the azimuth origin of
// the caps is e1 = e x z (or e x x when e is nearly parallel to z).
void frame(const double e[3], double e1[3], double e2[3]) {
  const double z[3] = {0, 0, 1}, x[3] = {1, 0, 0};
  cross(e, z, e1);
  if (norm3(e1) < 0.1) cross(e, x, e1);
  double n = norm3(e1);
  for (int i = 0; i < 3; ++i) e1[i] /= n;
  cross(e, e1, e2);
}

// Cap node j (1-based) of an m-node cap: local (cos t, sin t cos p, sin t sin p).
inline void cap_node(int j, int m, double beta, bool shifted, double loc[3]) {
  double jt = shifted ? j - 0.5 : j;
  double ct = 1.0 - jt * (1.0 - std::cos(beta)) / m;
  double st = std::sqrt(std::fmax(0.0, 1.0 - ct * ct));
  double jp = shifted ? j + 0.5 : j;
  double ph = std::fmod(2.0 * kPi * jp / golden(), 2.0 * kPi);
  loc[0] = ct;
  loc[1] = st * std::cos(ph);
  loc[2] = st * std::sin(ph);
}

double racc(double d) { return 1.0 + 0.5 * d - std::sqrt(d + 0.25 * d * d); }

int image_rule(double d) {
  if (d < 0.15) return (int)std::ceil(-8.72 * std::log10(d) - 6.15);
  return 0;
}

void push3(std::vector<double> &v, double x, double y, double z) {
  v.push_back(x);
  v.push_back(y);
  v.push_back(z);
}

}  // namespace

int build_geometry(Problem &pb) {
  const smfs_params &p = pb.prm;
  const int P = pb.P;
  const double a = pb.a;
  pb.contacts.assign(P, {});
  pb.n_contacts = 0;
  pb.small_gap = false;
  for (int k = 0; k < P; ++k) {
    const double *ck = &pb.centers[3 * k];
    for (int o = 0; o < P; ++o) {
      if (o == k) continue;
      const double *co = &pb.centers[3 * o];
      double d[3] = {co[0] - ck[0], co[1] - ck[1], co[2] - ck[2]};
      double dist = norm3(d);
      double gap = dist / a - 2.0;
      if (!(gap > 0.0)) {
        set_error("spheres " + std::to_string(k) + " and " + std::to_string(o) + " overlap");
        return SMFS_E_OVERLAP;
      }
      if (gap < 1e-3) pb.small_gap = true;
      if (gap < p.image_gap_cutoff) {
        int nim = p.n_image >= 0 ? p.n_image : image_rule(gap);
        if (nim <= 0) continue;
        Contact c;
        c.other = o;
        c.gap = gap;
        for (int i = 0; i < 3; ++i) c.axis[i] = d[i] / dist;
        c.n_im = nim;
        pb.contacts[k].push_back(c);
        ++pb.n_contacts;
      }
    }
  }

  const bool kS = p.image_kinds & SMFS_KIND_S, kR = p.image_kinds & SMFS_KIND_R,
             kD = p.image_kinds & SMFS_KIND_D;
  pb.tgt.clear(); pb.tw.clear(); pb.tsph.clear(); pb.toff.assign(1, 0);
  pb.chk.clear(); pb.csph.clear();
  // blocks: 0 proxy Stokeslets, 1 image Stokeslets, 2 rotlets, 3 dipoles
  std::vector<double> spos[kBlocks];
  std::vector<int32_t> scount[kBlocks];
  for (int b = 0; b < kBlocks; ++b) scount[b].assign(P, 0);

  const double w_base = 4.0 * kPi * a * a / p.n_colloc_base;
  for (int k = 0; k < P; ++k) {
    const double *c = &pb.centers[3 * k];
    double u[3];
    for (int j = 1; j <= p.n_colloc_base; ++j) {
      spiral(j, p.n_colloc_base, 0.0, u);
      push3(pb.tgt, c[0] + a * u[0], c[1] + a * u[1], c[2] + a * u[2]);
      pb.tw.push_back(w_base);
      pb.tsph.push_back(k);
    }
    for (int j = 1; j <= p.n_check_base; ++j) {
      spiral(j, p.n_check_base, 0.5, u);
      push3(pb.chk, c[0] + a * u[0], c[1] + a * u[1], c[2] + a * u[2]);
      pb.csph.push_back(k);
    }
    const double rp = p.proxy_radius * a;
    for (int j = 1; j <= p.n_proxy; ++j) {
      spiral(j, p.n_proxy, 0.0, u);
      push3(spos[0], c[0] + rp * u[0], c[1] + rp * u[1], c[2] + rp * u[2]);
      scount[0][k]++;
    }
    for (const Contact &ct : pb.contacts[k]) {
      const double t0 = p.proxy_radius * (1.0 + p.image_offset);
      const double ra = racc(ct.gap);
      for (int j = 1; j <= ct.n_im; ++j) {
        double t = t0 + (ra - t0) * std::cos((j - 1.0) * kPi / (2.0 * ct.n_im));
        double x = c[0] + a * t * ct.axis[0], y = c[1] + a * t * ct.axis[1],
               z = c[2] + a * t * ct.axis[2];
        if (kS) { push3(spos[1], x, y, z); scount[1][k]++; }
        if (kR) { push3(spos[2], x, y, z); scount[2][k]++; }
        if (kD) { push3(spos[3], x, y, z); scount[3][k]++; }
      }
      double e1[3], e2[3];
      frame(ct.axis, e1, e2);
      for (int cap = 0; cap < 2; ++cap) {
        const int m = p.cap_alpha[cap] * 3 * ct.n_im;
        const double beta = p.cap_beta[cap];
        const double w = 2.0 * kPi * a * a * (1.0 - std::cos(beta)) / m;
        for (int pass = 0; pass < 2; ++pass) {
          for (int j = 1; j <= m; ++j) {
            double loc[3];
            cap_node(j, m, beta, pass == 1, loc);
            double v[3];
            for (int i = 0; i < 3; ++i) v[i] = loc[0] * ct.axis[i] + loc[1] * e1[i] + loc[2] * e2[i];
            if (pass == 0) {
              push3(pb.tgt, c[0] + a * v[0], c[1] + a * v[1], c[2] + a * v[2]);
              pb.tw.push_back(w);
              pb.tsph.push_back(k);
            } else {
              push3(pb.chk, c[0] + a * v[0], c[1] + a * v[1], c[2] + a * v[2]);
              pb.csph.push_back(k);
            }
          }
        }
      }
    }
    pb.toff.push_back((int64_t)pb.tsph.size());
  }
  pb.T = (int64_t)pb.tsph.size();
  pb.C = (int64_t)pb.csph.size();

  // pack sources block by block, sphere-major inside each block
  static const int kBlockKind[kBlocks] = {0, 0, 1, 2};
  pb.src.clear(); pb.skind.clear(); pb.ssph.clear();
  int64_t base = 0;
  for (int b = 0; b < kBlocks; ++b) {
    pb.koff[b].assign(P + 1, 0);
    pb.koff[b][0] = base;
    int64_t pos = 0;
    for (int k = 0; k < P; ++k) {
      for (int j = 0; j < scount[b][k]; ++j, ++pos) {
        push3(pb.src, spos[b][3 * pos], spos[b][3 * pos + 1], spos[b][3 * pos + 2]);
        pb.skind.push_back(kBlockKind[b]);
        pb.ssph.push_back(k);
      }
      base += scount[b][k];
      pb.koff[b][k + 1] = base;
    }
    pb.nb[b] = pb.koff[b][P] - pb.koff[b][0];
  }
  pb.nk[0] = pb.nb[0] + pb.nb[1];
  pb.nk[1] = pb.nb[2];
  pb.nk[2] = pb.nb[3];
  pb.S = base;

  // factor ids: 0 for every contact-free sphere, then one per contact sphere
  pb.fid_of.assign(P, 0);
  pb.factors.clear();
  bool any_free = false;
  int nf = 1;
  for (int k = 0; k < P; ++k) {
    if (pb.contacts[k].empty()) any_free = true;
    else pb.fid_of[k] = nf++;
  }
  pb.factors.resize(nf);
  for (int f = 0; f < nf; ++f) pb.factors[f].rep = -1;
  for (int k = 0; k < P; ++k)
    if (pb.factors[pb.fid_of[k]].rep < 0) pb.factors[pb.fid_of[k]].rep = k;
  if (!any_free) pb.factors[0].rep = -1;  // slot 0 unused
  for (int f = 0; f < nf; ++f) {
    FactorSlot &fs = pb.factors[f];
    fs.rank = 0;
    if (fs.rep < 0) { fs.rows = fs.cols = 0; continue; }
    int k = fs.rep;
    fs.rows = (int32_t)(3 * (pb.toff[k + 1] - pb.toff[k]));
    int64_t n = 0;
    for (int b = 0; b < kBlocks; ++b) n += pb.koff[b][k + 1] - pb.koff[b][k];
    fs.cols = (int32_t)(3 * n);
  }
  // pairs per apply: every collocation node against every source of other spheres
  pb.pairs_per_apply = 0;
  pb.pairs_f32 = 0;
  for (int kd = 0; kd < 3; ++kd) pb.pairs_kind[kd] = 0;
  int64_t free_proxies = 0;
  for (int k = 0; k < P; ++k)
    if (pb.contacts[k].empty()) free_proxies += pb.koff[0][k + 1] - pb.koff[0][k];
  for (int k = 0; k < P; ++k) {
    const int64_t Mk = pb.toff[k + 1] - pb.toff[k];
    for (int b = 0; b < kBlocks; ++b)
      pb.pairs_kind[kBlockKind[b]] += Mk * (pb.nb[b] - (pb.koff[b][k + 1] - pb.koff[b][k]));
    const int64_t own = pb.contacts[k].empty() ? pb.koff[0][k + 1] - pb.koff[0][k] : 0;
    pb.pairs_f32 += Mk * (free_proxies - own);
  }
  pb.pairs_per_apply = pb.pairs_kind[0] + pb.pairs_kind[1] + pb.pairs_kind[2];
  return SMFS_OK;
}

// n points of the Fibonacci spiral on the sphere of radius r about the
// origin (the proxies' spiral), n x 3.
void spiral_points(int n, double r, std::vector<double> &out) {
  out.assign(3 * (size_t)n, 0.0);
  for (int j = 1; j <= n; ++j) {
    double u[3];
    spiral(j, n, 0.0, u);
    for (int c = 0; c < 3; ++c) out[3 * (size_t)(j - 1) + c] = r * u[c];
  }
}

// Near lists of the equivalent-source far field: for every sphere k, the
// contact-free spheres k' != k (as free indices, ascending) whose centres
// lie closer than sep; the pair counts of the SMFS_MIXED_EQ product.
// Spheres are swept in order of x, so only candidates within sep in x are
// tested.
void build_near_lists(Problem &pb, double sep) {
  const int P = pb.P;
  std::vector<int32_t> free_of(P, -1);
  int32_t nf = 0;
  for (int k = 0; k < P; ++k)
    if (pb.contacts[k].empty()) free_of[k] = nf++;
  std::vector<int> ord(P);
  for (int k = 0; k < P; ++k) ord[k] = k;
  std::sort(ord.begin(), ord.end(), [&](int x, int y) { return pb.centers[3 * x] < pb.centers[3 * y]; });
  std::vector<std::vector<int32_t>> lists(P);
  const double s2 = sep * sep;
  for (int a = 0; a < P; ++a) {
    const int k = ord[a];
    const double *ck = &pb.centers[3 * k];
    for (int b = a + 1; b < P; ++b) {
      const int ks = ord[b];
      const double *cs = &pb.centers[3 * ks];
      if (cs[0] - ck[0] >= sep) break;
      const double dx = ck[0] - cs[0], dy = ck[1] - cs[1], dz = ck[2] - cs[2];
      if (dx * dx + dy * dy + dz * dz >= s2) continue;
      if (free_of[ks] >= 0) lists[k].push_back(free_of[ks]);
      if (free_of[k] >= 0) lists[ks].push_back(free_of[k]);
    }
  }
  pb.near_off.assign(P + 1, 0);
  pb.near_idx.clear();
  pb.pairs_eq_far = pb.pairs_eq_exact = 0;
  for (int k = 0; k < P; ++k) {
    std::sort(lists[k].begin(), lists[k].end());
    pb.near_idx.insert(pb.near_idx.end(), lists[k].begin(), lists[k].end());
    pb.near_off[k + 1] = (int32_t)pb.near_idx.size();
    const int64_t Mk = pb.toff[k + 1] - pb.toff[k];
    const int64_t far = nf - (free_of[k] >= 0 ? 1 : 0) - (int64_t)lists[k].size();
    pb.pairs_eq_far += Mk * far * pb.n_eq;
    pb.pairs_eq_exact += Mk * far * pb.prm.n_proxy;   // subtracted below
  }
  pb.pairs_eq_exact = pb.pairs_per_apply - pb.pairs_eq_exact;
}

}  // namespace smfs
