/* Oracle direct sum (test infrastructure; plain C, float64, OpenMP over
 * targets).  Shares nothing with the HIP library.
 *
 *   u(x_i) = sum_j K_j(x_i - y_j) lam_j
 *
 * with K_j the Stokeslet (kind 0), rotlet (kind 1) or potential dipole
 * (kind 2) of the paper's Section 2.3:
 *   S(r) f = (f + r (r.f)/|r|^2) / (8 pi mu |r|)
 *   R(r) t = (t x r) / (8 pi mu |r|^3)
 *   D(r) d = (-d/|r|^3 + 3 r (r.d)/|r|^5) / (4 pi)
 * When skip_same is non-zero, source j is left out for target i whenever
 * they belong to the same sphere (the identity diagonal blocks of the
 * one-body preconditioned operator, Section 2.2).
 * Arrays are row-major: x (nt x 3), y (ns x 3), lam (ns x 3), u (nt x 3).
 */
#include <math.h>
#include <stdint.h>

void oracle_pairsum(int64_t nt, const double *x, const int32_t *tsph,
                    int64_t ns, const double *y, const int32_t *kind,
                    const int32_t *ssph, const double *lam, double mu,
                    int skip_same, double *u)
{
    const double pi = 3.14159265358979323846;
    const double cS = 1.0 / (8.0 * pi * mu);
    const double cD = 1.0 / (4.0 * pi);
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < nt; ++i) {
        double ux = 0.0, uy = 0.0, uz = 0.0;
        double xi0 = x[3 * i], xi1 = x[3 * i + 1], xi2 = x[3 * i + 2];
        int32_t si = tsph ? tsph[i] : -1;
        int64_t j;
        for (j = 0; j < ns; ++j) {
            if (skip_same && ssph[j] == si)
                continue;
            double r0 = xi0 - y[3 * j], r1 = xi1 - y[3 * j + 1], r2 = xi2 - y[3 * j + 2];
            double rr = r0 * r0 + r1 * r1 + r2 * r2;
            double rn = sqrt(rr);
            double l0 = lam[3 * j], l1 = lam[3 * j + 1], l2 = lam[3 * j + 2];
            if (kind[j] == 0) {
                double rl = r0 * l0 + r1 * l1 + r2 * l2;
                double a = cS / rn, b = cS * rl / (rr * rn);
                ux += a * l0 + b * r0;
                uy += a * l1 + b * r1;
                uz += a * l2 + b * r2;
            } else if (kind[j] == 1) {
                double c = cS / (rr * rn);
                ux += c * (l1 * r2 - l2 * r1);
                uy += c * (l2 * r0 - l0 * r2);
                uz += c * (l0 * r1 - l1 * r0);
            } else {
                double rl = r0 * l0 + r1 * l1 + r2 * l2;
                double r3 = rr * rn;
                double a = -cD / r3, b = 3.0 * cD * rl / (r3 * rr);
                ux += a * l0 + b * r0;
                uy += a * l1 + b * r1;
                uz += a * l2 + b * r2;
            }
        }
        u[3 * i] = ux;
        u[3 * i + 1] = uy;
        u[3 * i + 2] = uz;
    }
}
