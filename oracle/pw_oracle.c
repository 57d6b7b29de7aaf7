/*
 * Piacsek-Williams (PW) advection: plain FP64 reference ("the oracle").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct CPU
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header or table with the HIP
 * library.
 *
 * What is computed (paper, Sec. 2.2 and Sec. 4):
 *   Three wind fields u, v, w (x, y and z velocity) are advected by
 *   themselves.  For every interior grid cell the scheme produces one
 *   "source term" per field (su, sv, sw) from a depth-one stencil that
 *   reaches the neighbouring cells in all three dimensions.  Per field and
 *   cell the paper counts six additions, six multiplications, then
 *   subtractions and an addition reduction (Sec. 4, Fig. 2), with the same
 *   arithmetic for all three fields and only the stencil locations differing.
 *
 * The paper does not print the equations.  The reading used here is the
 * energy-conserving PW form on a staggered (Arakawa C) grid, as used in the
 * MONC model the paper takes the kernel from:  u sits on east faces
 * (i+1/2), v on north faces (j+1/2), w on top faces (k+1/2); each term is a
 * coefficient times a neighbouring value of the advected field times the sum
 * of two advecting-velocity values at the shared face, upstream face minus
 * downstream face.  tcx, tcy are scalars; tzc1/tzc2 (u, v) and tzd1/tzd2 (w)
 * are per-level arrays, 1 = lower face, 2 = upper face.
 *
 * Layout: every input is a dense C-order array of the halo-padded shape
 * (nz+2h, ny+2h, nx+2h), x fastest; indices below are padded coordinates,
 * interior k, j, i in [h, h+n).  Outputs are dense (nz, ny, nx).  The
 * vertical arrays have length nz and are indexed by the interior level k-h.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC.  No FMA
 * contraction, fixed term order.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IDX(k, j, i) ((((int64_t)(k)) * py + (int64_t)(j)) * px + (int64_t)(i))
#define U(k, j, i) u[IDX(k, j, i)]
#define V(k, j, i) v[IDX(k, j, i)]
#define W(k, j, i) w[IDX(k, j, i)]

/* Forward operator F: (u, v, w) -> (su, sv, sw) at every interior point.
 * If mag_* are non-NULL they receive A(p) = sum over the six products of
 * |coefficient| * |advected value| * (|face value 1| + |face value 2|), the
 * natural scale of the rounding error of any evaluation order. */
void pwo_forward(int64_t nx, int64_t ny, int64_t nz, int64_t h,
                 const double *u, const double *v, const double *w,
                 double tcx, double tcy,
                 const double *tzc1, const double *tzc2,
                 const double *tzd1, const double *tzd2,
                 double *su, double *sv, double *sw,
                 double *mag_u, double *mag_v, double *mag_w,
                 int nthreads)
{
    const int64_t px = nx + 2 * h, py = ny + 2 * h;
    if (nthreads < 1) nthreads = 1;
#ifdef _OPENMP
#pragma omp parallel for num_threads(nthreads) schedule(static)
#endif
    for (int64_t k = h; k < h + nz; ++k) {
        const int64_t kk = k - h;          /* interior level: vertical arrays */
        for (int64_t j = h; j < h + ny; ++j) {
            for (int64_t i = h; i < h + nx; ++i) {
                const int64_t o = (kk * ny + (j - h)) * nx + (i - h);
                double x, y, z;

                /* su: u advected through the x, y and z faces of the u cell */
                x = tcx * (U(k, j, i - 1) * (U(k, j, i) + U(k, j, i - 1))
                         - U(k, j, i + 1) * (U(k, j, i) + U(k, j, i + 1)));
                y = tcy * (U(k, j - 1, i) * (V(k, j - 1, i) + V(k, j - 1, i + 1))
                         - U(k, j + 1, i) * (V(k, j, i) + V(k, j, i + 1)));
                z = tzc1[kk] * U(k - 1, j, i) * (W(k - 1, j, i) + W(k - 1, j, i + 1))
                  - tzc2[kk] * U(k + 1, j, i) * (W(k, j, i) + W(k, j, i + 1));
                su[o] = x + y + z;

                /* sv: v advected through the x, y and z faces of the v cell */
                x = tcx * (V(k, j, i - 1) * (U(k, j, i - 1) + U(k, j + 1, i - 1))
                         - V(k, j, i + 1) * (U(k, j, i) + U(k, j + 1, i)));
                y = tcy * (V(k, j - 1, i) * (V(k, j, i) + V(k, j - 1, i))
                         - V(k, j + 1, i) * (V(k, j, i) + V(k, j + 1, i)));
                z = tzc1[kk] * V(k - 1, j, i) * (W(k - 1, j, i) + W(k - 1, j + 1, i))
                  - tzc2[kk] * V(k + 1, j, i) * (W(k, j, i) + W(k, j + 1, i));
                sv[o] = x + y + z;

                /* sw: w advected through the x, y and z faces of the w cell */
                x = tcx * (W(k, j, i - 1) * (U(k, j, i - 1) + U(k + 1, j, i - 1))
                         - W(k, j, i + 1) * (U(k, j, i) + U(k + 1, j, i)));
                y = tcy * (W(k, j - 1, i) * (V(k, j - 1, i) + V(k + 1, j - 1, i))
                         - W(k, j + 1, i) * (V(k, j, i) + V(k + 1, j, i)));
                z = tzd1[kk] * W(k - 1, j, i) * (W(k, j, i) + W(k - 1, j, i))
                  - tzd2[kk] * W(k + 1, j, i) * (W(k, j, i) + W(k + 1, j, i));
                sw[o] = x + y + z;

                if (mag_u) {
                    mag_u[o] = fabs(tcx) * fabs(U(k, j, i - 1)) * (fabs(U(k, j, i)) + fabs(U(k, j, i - 1)))
                             + fabs(tcx) * fabs(U(k, j, i + 1)) * (fabs(U(k, j, i)) + fabs(U(k, j, i + 1)))
                             + fabs(tcy) * fabs(U(k, j - 1, i)) * (fabs(V(k, j - 1, i)) + fabs(V(k, j - 1, i + 1)))
                             + fabs(tcy) * fabs(U(k, j + 1, i)) * (fabs(V(k, j, i)) + fabs(V(k, j, i + 1)))
                             + fabs(tzc1[kk]) * fabs(U(k - 1, j, i)) * (fabs(W(k - 1, j, i)) + fabs(W(k - 1, j, i + 1)))
                             + fabs(tzc2[kk]) * fabs(U(k + 1, j, i)) * (fabs(W(k, j, i)) + fabs(W(k, j, i + 1)));
                }
                if (mag_v) {
                    mag_v[o] = fabs(tcx) * fabs(V(k, j, i - 1)) * (fabs(U(k, j, i - 1)) + fabs(U(k, j + 1, i - 1)))
                             + fabs(tcx) * fabs(V(k, j, i + 1)) * (fabs(U(k, j, i)) + fabs(U(k, j + 1, i)))
                             + fabs(tcy) * fabs(V(k, j - 1, i)) * (fabs(V(k, j, i)) + fabs(V(k, j - 1, i)))
                             + fabs(tcy) * fabs(V(k, j + 1, i)) * (fabs(V(k, j, i)) + fabs(V(k, j + 1, i)))
                             + fabs(tzc1[kk]) * fabs(V(k - 1, j, i)) * (fabs(W(k - 1, j, i)) + fabs(W(k - 1, j + 1, i)))
                             + fabs(tzc2[kk]) * fabs(V(k + 1, j, i)) * (fabs(W(k, j, i)) + fabs(W(k, j + 1, i)));
                }
                if (mag_w) {
                    mag_w[o] = fabs(tcx) * fabs(W(k, j, i - 1)) * (fabs(U(k, j, i - 1)) + fabs(U(k + 1, j, i - 1)))
                             + fabs(tcx) * fabs(W(k, j, i + 1)) * (fabs(U(k, j, i)) + fabs(U(k + 1, j, i)))
                             + fabs(tcy) * fabs(W(k, j - 1, i)) * (fabs(V(k, j - 1, i)) + fabs(V(k + 1, j - 1, i)))
                             + fabs(tcy) * fabs(W(k, j + 1, i)) * (fabs(V(k, j, i)) + fabs(V(k + 1, j, i)))
                             + fabs(tzd1[kk]) * fabs(W(k - 1, j, i)) * (fabs(W(k, j, i)) + fabs(W(k - 1, j, i)))
                             + fabs(tzd2[kk]) * fabs(W(k + 1, j, i)) * (fabs(W(k, j, i)) + fabs(W(k + 1, j, i)));
                }
            }
        }
    }
}

/* One product term  s * c * a * (b + d)  with cotangent r contributes
 *   d/da = s*c*(b+d)*r,   d/db = d/dd = s*c*a*r
 * to the gradient.  ga, gb, gd point at the gradient entries of a, b, d. */
static void scatter_term(double s, double c, double r,
                         double *ga, double a, double *gb, double b, double *gd, double d)
{
    *ga += s * c * (b + d) * r;
    *gb += s * c * a * r;
    *gd += s * c * a * r;
}

#define GU(k, j, i) (&gu[IDX(k, j, i)])
#define GV(k, j, i) (&gv[IDX(k, j, i)])
#define GW(k, j, i) (&gw[IDX(k, j, i)])

/* Adjoint (vector-Jacobian product) of the forward operator:
 *   (gu, gv, gw) = J(u, v, w)^T (ru, rv, rw),
 * where ru, rv, rw are interior-shaped cotangents of su, sv, sw and the
 * gradients cover the whole padded arrays, halo included.  This is the plain
 * definition: for every interior point and every product term of every
 * output, the product rule is applied and the partials are added into the
 * entries the term reads.  gu, gv, gw are overwritten.  Serial on purpose
 * (the scatter would race under threads). */
void pwo_adjoint(int64_t nx, int64_t ny, int64_t nz, int64_t h,
                 const double *u, const double *v, const double *w,
                 double tcx, double tcy,
                 const double *tzc1, const double *tzc2,
                 const double *tzd1, const double *tzd2,
                 const double *ru, const double *rv, const double *rw,
                 double *gu, double *gv, double *gw)
{
    const int64_t px = nx + 2 * h, py = ny + 2 * h;
    const int64_t npad = px * py * (nz + 2 * h);
    for (int64_t q = 0; q < npad; ++q) { gu[q] = 0.0; gv[q] = 0.0; gw[q] = 0.0; }

    for (int64_t k = h; k < h + nz; ++k) {
        const int64_t kk = k - h;
        for (int64_t j = h; j < h + ny; ++j) {
            for (int64_t i = h; i < h + nx; ++i) {
                const int64_t o = (kk * ny + (j - h)) * nx + (i - h);
                double r;

                r = ru[o];   /* su */
                scatter_term(+1.0, tcx, r, GU(k, j, i - 1), U(k, j, i - 1),
                             GU(k, j, i), U(k, j, i), GU(k, j, i - 1), U(k, j, i - 1));
                scatter_term(-1.0, tcx, r, GU(k, j, i + 1), U(k, j, i + 1),
                             GU(k, j, i), U(k, j, i), GU(k, j, i + 1), U(k, j, i + 1));
                scatter_term(+1.0, tcy, r, GU(k, j - 1, i), U(k, j - 1, i),
                             GV(k, j - 1, i), V(k, j - 1, i), GV(k, j - 1, i + 1), V(k, j - 1, i + 1));
                scatter_term(-1.0, tcy, r, GU(k, j + 1, i), U(k, j + 1, i),
                             GV(k, j, i), V(k, j, i), GV(k, j, i + 1), V(k, j, i + 1));
                scatter_term(+1.0, tzc1[kk], r, GU(k - 1, j, i), U(k - 1, j, i),
                             GW(k - 1, j, i), W(k - 1, j, i), GW(k - 1, j, i + 1), W(k - 1, j, i + 1));
                scatter_term(-1.0, tzc2[kk], r, GU(k + 1, j, i), U(k + 1, j, i),
                             GW(k, j, i), W(k, j, i), GW(k, j, i + 1), W(k, j, i + 1));

                r = rv[o];   /* sv */
                scatter_term(+1.0, tcx, r, GV(k, j, i - 1), V(k, j, i - 1),
                             GU(k, j, i - 1), U(k, j, i - 1), GU(k, j + 1, i - 1), U(k, j + 1, i - 1));
                scatter_term(-1.0, tcx, r, GV(k, j, i + 1), V(k, j, i + 1),
                             GU(k, j, i), U(k, j, i), GU(k, j + 1, i), U(k, j + 1, i));
                scatter_term(+1.0, tcy, r, GV(k, j - 1, i), V(k, j - 1, i),
                             GV(k, j, i), V(k, j, i), GV(k, j - 1, i), V(k, j - 1, i));
                scatter_term(-1.0, tcy, r, GV(k, j + 1, i), V(k, j + 1, i),
                             GV(k, j, i), V(k, j, i), GV(k, j + 1, i), V(k, j + 1, i));
                scatter_term(+1.0, tzc1[kk], r, GV(k - 1, j, i), V(k - 1, j, i),
                             GW(k - 1, j, i), W(k - 1, j, i), GW(k - 1, j + 1, i), W(k - 1, j + 1, i));
                scatter_term(-1.0, tzc2[kk], r, GV(k + 1, j, i), V(k + 1, j, i),
                             GW(k, j, i), W(k, j, i), GW(k, j + 1, i), W(k, j + 1, i));

                r = rw[o];   /* sw */
                scatter_term(+1.0, tcx, r, GW(k, j, i - 1), W(k, j, i - 1),
                             GU(k, j, i - 1), U(k, j, i - 1), GU(k + 1, j, i - 1), U(k + 1, j, i - 1));
                scatter_term(-1.0, tcx, r, GW(k, j, i + 1), W(k, j, i + 1),
                             GU(k, j, i), U(k, j, i), GU(k + 1, j, i), U(k + 1, j, i));
                scatter_term(+1.0, tcy, r, GW(k, j - 1, i), W(k, j - 1, i),
                             GV(k, j - 1, i), V(k, j - 1, i), GV(k + 1, j - 1, i), V(k + 1, j - 1, i));
                scatter_term(-1.0, tcy, r, GW(k, j + 1, i), W(k, j + 1, i),
                             GV(k, j, i), V(k, j, i), GV(k + 1, j, i), V(k + 1, j, i));
                scatter_term(+1.0, tzd1[kk], r, GW(k - 1, j, i), W(k - 1, j, i),
                             GW(k, j, i), W(k, j, i), GW(k - 1, j, i), W(k - 1, j, i));
                scatter_term(-1.0, tzd2[kk], r, GW(k + 1, j, i), W(k + 1, j, i),
                             GW(k, j, i), W(k, j, i), GW(k + 1, j, i), W(k + 1, j, i));
            }
        }
    }
}

/* Tangent-linear operator (Jacobian-vector product):
 *   (tu, tv, tw) = J(u, v, w) (du, dv, dw),
 * the directional derivative of every output along the padded direction
 * (du, dv, dw).  Each product term s*c*a*(b+d) differentiates to
 * s*c*(da*(b+d) + a*(db+dd)).  Outputs are interior-shaped. */
#define DU(k, j, i) du[IDX(k, j, i)]
#define DV(k, j, i) dv[IDX(k, j, i)]
#define DW(k, j, i) dw[IDX(k, j, i)]
#define TL(a, da, b, db, d, dd) ((da) * ((b) + (d)) + (a) * ((db) + (dd)))

void pwo_tangent(int64_t nx, int64_t ny, int64_t nz, int64_t h,
                 const double *u, const double *v, const double *w,
                 const double *du, const double *dv, const double *dw,
                 double tcx, double tcy,
                 const double *tzc1, const double *tzc2,
                 const double *tzd1, const double *tzd2,
                 double *tu, double *tv, double *tw)
{
    const int64_t px = nx + 2 * h, py = ny + 2 * h;
    for (int64_t k = h; k < h + nz; ++k) {
        const int64_t kk = k - h;
        for (int64_t j = h; j < h + ny; ++j) {
            for (int64_t i = h; i < h + nx; ++i) {
                const int64_t o = (kk * ny + (j - h)) * nx + (i - h);
                tu[o] = tcx * (TL(U(k, j, i - 1), DU(k, j, i - 1), U(k, j, i), DU(k, j, i), U(k, j, i - 1), DU(k, j, i - 1))
                             - TL(U(k, j, i + 1), DU(k, j, i + 1), U(k, j, i), DU(k, j, i), U(k, j, i + 1), DU(k, j, i + 1)))
                      + tcy * (TL(U(k, j - 1, i), DU(k, j - 1, i), V(k, j - 1, i), DV(k, j - 1, i), V(k, j - 1, i + 1), DV(k, j - 1, i + 1))
                             - TL(U(k, j + 1, i), DU(k, j + 1, i), V(k, j, i), DV(k, j, i), V(k, j, i + 1), DV(k, j, i + 1)))
                      + tzc1[kk] * TL(U(k - 1, j, i), DU(k - 1, j, i), W(k - 1, j, i), DW(k - 1, j, i), W(k - 1, j, i + 1), DW(k - 1, j, i + 1))
                      - tzc2[kk] * TL(U(k + 1, j, i), DU(k + 1, j, i), W(k, j, i), DW(k, j, i), W(k, j, i + 1), DW(k, j, i + 1));
                tv[o] = tcx * (TL(V(k, j, i - 1), DV(k, j, i - 1), U(k, j, i - 1), DU(k, j, i - 1), U(k, j + 1, i - 1), DU(k, j + 1, i - 1))
                             - TL(V(k, j, i + 1), DV(k, j, i + 1), U(k, j, i), DU(k, j, i), U(k, j + 1, i), DU(k, j + 1, i)))
                      + tcy * (TL(V(k, j - 1, i), DV(k, j - 1, i), V(k, j, i), DV(k, j, i), V(k, j - 1, i), DV(k, j - 1, i))
                             - TL(V(k, j + 1, i), DV(k, j + 1, i), V(k, j, i), DV(k, j, i), V(k, j + 1, i), DV(k, j + 1, i)))
                      + tzc1[kk] * TL(V(k - 1, j, i), DV(k - 1, j, i), W(k - 1, j, i), DW(k - 1, j, i), W(k - 1, j + 1, i), DW(k - 1, j + 1, i))
                      - tzc2[kk] * TL(V(k + 1, j, i), DV(k + 1, j, i), W(k, j, i), DW(k, j, i), W(k, j + 1, i), DW(k, j + 1, i));
                tw[o] = tcx * (TL(W(k, j, i - 1), DW(k, j, i - 1), U(k, j, i - 1), DU(k, j, i - 1), U(k + 1, j, i - 1), DU(k + 1, j, i - 1))
                             - TL(W(k, j, i + 1), DW(k, j, i + 1), U(k, j, i), DU(k, j, i), U(k + 1, j, i), DU(k + 1, j, i)))
                      + tcy * (TL(W(k, j - 1, i), DW(k, j - 1, i), V(k, j - 1, i), DV(k, j - 1, i), V(k + 1, j - 1, i), DV(k + 1, j - 1, i))
                             - TL(W(k, j + 1, i), DW(k, j + 1, i), V(k, j, i), DV(k, j, i), V(k + 1, j, i), DV(k + 1, j, i)))
                      + tzd1[kk] * TL(W(k - 1, j, i), DW(k - 1, j, i), W(k, j, i), DW(k, j, i), W(k - 1, j, i), DW(k - 1, j, i))
                      - tzd2[kk] * TL(W(k + 1, j, i), DW(k + 1, j, i), W(k, j, i), DW(k, j, i), W(k + 1, j, i), DW(k + 1, j, i));
            }
        }
    }
}

/* Gradients of L = <su, ru> + <sv, rv> + <sw, rw> with respect to the
 * coefficients.  Every term of the operator is one coefficient times a
 * coefficient-free product, so dL/dc is the sum, over the terms that c
 * multiplies, of the cotangent at the term's output times that product:
 *   gtcx        = sum over all points of the x-face products (u, v, w rows)
 *   gtcy        = the same for the y-face products
 *   gtzc1[k]    = sum over level k of ru*u(k-1)*(w+w at k-1) + rv*v(k-1)*(...)
 *   gtzc2[k]    = minus the same for the upper faces
 *   gtzd1/2[k]  = the w field's lower / upper face products times rw.
 * gtcx_lev[k] and gtcy_lev[k] receive level k's share of gtcx and gtcy. */
void pwo_coeff_grad(int64_t nx, int64_t ny, int64_t nz, int64_t h,
                    const double *u, const double *v, const double *w,
                    const double *ru, const double *rv, const double *rw,
                    double *gtzc1, double *gtzc2, double *gtzd1, double *gtzd2,
                    double *gtcx_lev, double *gtcy_lev, double *gtcx, double *gtcy)
{
    const int64_t px = nx + 2 * h, py = ny + 2 * h;
    double sx = 0.0, sy = 0.0;
    for (int64_t k = h; k < h + nz; ++k) {
        const int64_t kk = k - h;
        double c1 = 0.0, c2 = 0.0, d1 = 0.0, d2 = 0.0, lx = 0.0, ly = 0.0;
        for (int64_t j = h; j < h + ny; ++j) {
            for (int64_t i = h; i < h + nx; ++i) {
                const int64_t o = (kk * ny + (j - h)) * nx + (i - h);
                const double a = ru[o], b = rv[o], c = rw[o];
                /* su */
                lx += a * (U(k, j, i - 1) * (U(k, j, i) + U(k, j, i - 1)) - U(k, j, i + 1) * (U(k, j, i) + U(k, j, i + 1)));
                ly += a * (U(k, j - 1, i) * (V(k, j - 1, i) + V(k, j - 1, i + 1)) - U(k, j + 1, i) * (V(k, j, i) + V(k, j, i + 1)));
                c1 += a * (U(k - 1, j, i) * (W(k - 1, j, i) + W(k - 1, j, i + 1)));
                c2 -= a * (U(k + 1, j, i) * (W(k, j, i) + W(k, j, i + 1)));
                /* sv */
                lx += b * (V(k, j, i - 1) * (U(k, j, i - 1) + U(k, j + 1, i - 1)) - V(k, j, i + 1) * (U(k, j, i) + U(k, j + 1, i)));
                ly += b * (V(k, j - 1, i) * (V(k, j, i) + V(k, j - 1, i)) - V(k, j + 1, i) * (V(k, j, i) + V(k, j + 1, i)));
                c1 += b * (V(k - 1, j, i) * (W(k - 1, j, i) + W(k - 1, j + 1, i)));
                c2 -= b * (V(k + 1, j, i) * (W(k, j, i) + W(k, j + 1, i)));
                /* sw */
                lx += c * (W(k, j, i - 1) * (U(k, j, i - 1) + U(k + 1, j, i - 1)) - W(k, j, i + 1) * (U(k, j, i) + U(k + 1, j, i)));
                ly += c * (W(k, j - 1, i) * (V(k, j - 1, i) + V(k + 1, j - 1, i)) - W(k, j + 1, i) * (V(k, j, i) + V(k + 1, j, i)));
                d1 += c * (W(k - 1, j, i) * (W(k, j, i) + W(k - 1, j, i)));
                d2 -= c * (W(k + 1, j, i) * (W(k, j, i) + W(k + 1, j, i)));
            }
        }
        gtzc1[kk] = c1;
        gtzc2[kk] = c2;
        gtzd1[kk] = d1;
        gtzd2[kk] = d2;
        gtcx_lev[kk] = lx;
        gtcy_lev[kk] = ly;
        sx += lx;
        sy += ly;
    }
    *gtcx = sx;
    *gtcy = sy;
}
