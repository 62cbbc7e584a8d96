/*
 * ddo.c -- plain, slow, single-threaded FP64 oracle for the DD pair-force hot
 * path.  TEST INFRASTRUCTURE ONLY: the product library never links, loads or
 * calls anything in this directory; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark do.
 *
 * What it computes (every function names the passage it follows):
 *
 *  - the stress of a straight dislocation segment, from the paper's statement
 *    that the stress of a loop is a differential operator acting on the
 *    distance R = x - x' convolved with the dislocation density (Sec. 2.1,
 *    "Discrete Dislocation Dynamics"), taken in its isotropic line-integral form
 *    with R replaced by R_a = sqrt(R.R + a^2) (non-singular, core width a), and
 *    integrated in closed form along the straight segment;
 *  - the Peach-Koehler force df_k = eps_kjm sigma_ji b_i dl_m (Sec. 2.1);
 *  - Q-point Gauss-Legendre quadrature of that force against the linear shape
 *    functions of each segment, scattered to its two nodes; optionally, for
 *    pairs inside a band around the target (the exact band, set by
 *    ddo_set_exact_band), the same integral along the target taken exactly
 *    (adaptive quadrature to rounding level) instead;
 *  - the glide-constrained linear mobility (velocity weak form, Eq. DD_evol:
 *    scalar drag, lumped, no-climb by projection onto the glide plane) and the
 *    forward-Euler node update (Sec. 2.1);
 *  - the per-slip-system plastic distortion rate b/A (x) (l x V), volume
 *    averaged (Sec. 2.2 "Thermal activation"), resolved on the 12 FCC systems
 *    and running-averaged over a burst with equal steps (Eq. R_lambda_t);
 *  - resolved shear stresses (the numerator of Eq. schmid) and per-system
 *    mobile/sessile densities (line length per volume, Sec. 2.4 item 2).
 *
 * Units: any consistent set.  Lengths (x, b, a) share a unit, mu and sigma share
 * a stress unit, B is stress*time and dt is time.  Forces come out in
 * stress*length^2.
 *
 * Layouts: x [3][n_nodes], seg_nodes [2][n_segs] (int32), burgers and normal
 * [3][n_segs], pinned [n_nodes] (uint8), sigma_app Voigt (xx,yy,zz,yz,xz,xy).
 *
 * No code here is shared with the HIP library; the arithmetic is arranged as
 * the plain formula (full 3x3 tensors, symmetric products written out), not as
 * the regrouped form the kernels use.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double mu, nu, a, B; } ddo_material;

#define DDO_MAX_Q 64
#define DDO_PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* small vector helpers                                                      */
/* ------------------------------------------------------------------------- */
static double dot3(const double *u, const double *v) { return u[0]*v[0] + u[1]*v[1] + u[2]*v[2]; }
static void cross3(const double *u, const double *v, double *w)
{
    w[0] = u[1]*v[2] - u[2]*v[1];
    w[1] = u[2]*v[0] - u[0]*v[2];
    w[2] = u[0]*v[1] - u[1]*v[0];
}
static void sym_add(double S[3][3], double coef, const double *p, const double *r)
{   /* S += coef * (p (x) r + r (x) p) */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            S[i][j] += coef * (p[i]*r[j] + r[i]*p[j]);
}
static void outer_add(double S[3][3], double coef, const double *p, const double *r)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            S[i][j] += coef * p[i]*r[j];
}
static void voigt_to_full(const double v[6], double S[3][3])
{
    S[0][0] = v[0]; S[1][1] = v[1]; S[2][2] = v[2];
    S[1][2] = S[2][1] = v[3];
    S[0][2] = S[2][0] = v[4];
    S[0][1] = S[1][0] = v[5];
}

/* ------------------------------------------------------------------------- */
/* Gauss-Legendre rule on [0,1]: nodes are the roots of the Legendre         */
/* polynomial P_n (three-term recurrence), found by Newton iteration from    */
/* the Chebyshev-like first guess cos(pi (i - 1/4)/(n + 1/2)); weights are   */
/* 2 / ((1 - z^2) P_n'(z)^2), halved for the map z -> s = (1 + z)/2.         */
/* ------------------------------------------------------------------------- */
int ddo_gauss_legendre(int n, double *s, double *w)
{
    if (n < 1 || n > DDO_MAX_Q) return -1;
    for (int i = 0; i < n; ++i) {
        double z = cos(DDO_PI * (i + 0.75) / (n + 0.5));
        double pn = 0.0, pm = 0.0;
        for (int it = 0; it < 100; ++it) {
            /* P_n(z) and P_{n-1}(z) by the three-term recurrence */
            pm = 1.0; pn = z;
            for (int k = 2; k <= n; ++k) {
                double pk = ((2.0*k - 1.0) * z * pn - (k - 1.0) * pm) / k;
                pm = pn; pn = pk;
            }
            double dp = n * (z * pn - pm) / (z*z - 1.0);
            double dz = pn / dp;
            z -= dz;
            if (fabs(dz) <= 1e-15 * fabs(z) + 1e-300) break;
        }
        pm = 1.0; pn = z;
        for (int k = 2; k <= n; ++k) {
            double pk = ((2.0*k - 1.0) * z * pn - (k - 1.0) * pm) / k;
            pm = pn; pn = pk;
        }
        double dp = n * (z * pn - pm) / (z*z - 1.0);
        /* z decreases with i: store ascending in s */
        s[n - 1 - i] = 0.5 * (1.0 + z);
        w[n - 1 - i] = 1.0 / ((1.0 - z*z) * dp * dp);
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Integrand: stress at R = x - x' from a unit length of straight line with  */
/* tangent t and Burgers vector b (isotropic line-integral form, R -> R_a).  */
/*  K = (mu/8pi) [-(2/Ra^3 + 3a^2/Ra^5)] [(R x b) (x) t + t (x) (R x b)]     */
/*    + (mu/(4pi(1-nu))) [ q (1/Ra^3 + 3a^2/Ra^5) I                          */
/*                         - (R (x) c + c (x) R)/Ra^3 + 3 q R (x) R / Ra^5 ] */
/*  with c = b x t and q = c.R.                                              */
/* ------------------------------------------------------------------------- */
void ddo_kernel(const double R[3], const double b[3], const double t[3],
                double mu, double nu, double a, double K[9])
{
    double S[3][3] = {{0}};
    double Ra2 = dot3(R, R) + a*a;
    double Ra = sqrt(Ra2);
    double Ra3 = Ra2 * Ra, Ra5 = Ra3 * Ra2;
    double Rxb[3], c[3];
    cross3(R, b, Rxb);
    cross3(b, t, c);
    double q = dot3(c, R);
    double k1 = mu / (8.0 * DDO_PI);
    double k2 = mu / (4.0 * DDO_PI * (1.0 - nu));
    sym_add(S, -k1 * (2.0/Ra3 + 3.0*a*a/Ra5), Rxb, t);
    for (int i = 0; i < 3; ++i) S[i][i] += k2 * q * (1.0/Ra3 + 3.0*a*a/Ra5);
    sym_add(S, -k2 / Ra3, R, c);
    outer_add(S, 3.0 * k2 * q / Ra5, R, R);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) K[3*i + j] = S[i][j];
}

/* ------------------------------------------------------------------------- */
/* Closed-form integral of the kernel along the straight segment x1 -> x2.   */
/* Write R0 = x - x1, t = (x2 - x1)/L, y = R0.t, rho = R0 - y t,             */
/* d2 = rho.rho + a^2 and u = s - y, so R = rho - u t and Ra^2 = d2 + u^2.   */
/* The integrals I_{n,k} = int u^k / Ra^n du over u in [-y, L - y] are       */
/*   J_{3,0} = u/(d2 Ra)           J_{3,1} = -1/Ra                           */
/*   J_{5,0} = u(2u^2+3d2)/(3 d2^2 Ra^3)                                     */
/*   J_{5,1} = -1/(3 Ra^3)         J_{5,2} = u^3/(3 d2 Ra^3)                 */
/* evaluated at both ends.  Substituting R = rho - u t into the integrand    */
/* and using c.t = 0 (so q = c.rho is constant along the segment):           */
/*   sigma = -(mu/8pi) [g0 S(rho x b, t) - g1 S(t x b, t)]                   */
/*         + (mu/(4pi(1-nu))) ( q (I30 + 3a^2 I50) I                         */
/*              - [I30 S(rho, c) - I31 S(t, c)]                              */
/*              + 3q [I50 rho(x)rho - I51 S(rho, t) + I52 t(x)t] )           */
/* with g0 = 2 I30 + 3a^2 I50, g1 = 2 I31 + 3a^2 I51, S(p,r) = p(x)r + r(x)p.*/
/* ------------------------------------------------------------------------- */
void ddo_segment_stress(const double x[3], const double x1[3], const double x2[3],
                        const double b[3], double mu, double nu, double a,
                        double sig[9])
{
    double d[3] = { x2[0]-x1[0], x2[1]-x1[1], x2[2]-x1[2] };
    double L = sqrt(dot3(d, d));
    double t[3] = { d[0]/L, d[1]/L, d[2]/L };
    double R0[3] = { x[0]-x1[0], x[1]-x1[1], x[2]-x1[2] };
    double y = dot3(R0, t);
    double rho[3] = { R0[0] - y*t[0], R0[1] - y*t[1], R0[2] - y*t[2] };
    double d2 = dot3(rho, rho) + a*a;
    double u1 = -y, u2 = L - y;
    double Ra1 = sqrt(d2 + u1*u1), Ra2 = sqrt(d2 + u2*u2);

    double J30_1 = u1 / (d2 * Ra1), J30_2 = u2 / (d2 * Ra2);
    double J31_1 = -1.0 / Ra1,      J31_2 = -1.0 / Ra2;
    double J50_1 = u1 * (2.0*u1*u1 + 3.0*d2) / (3.0 * d2*d2 * Ra1*Ra1*Ra1);
    double J50_2 = u2 * (2.0*u2*u2 + 3.0*d2) / (3.0 * d2*d2 * Ra2*Ra2*Ra2);
    double J51_1 = -1.0 / (3.0 * Ra1*Ra1*Ra1), J51_2 = -1.0 / (3.0 * Ra2*Ra2*Ra2);
    double J52_1 = u1*u1*u1 / (3.0 * d2 * Ra1*Ra1*Ra1);
    double J52_2 = u2*u2*u2 / (3.0 * d2 * Ra2*Ra2*Ra2);

    double I30 = J30_2 - J30_1, I31 = J31_2 - J31_1;
    double I50 = J50_2 - J50_1, I51 = J51_2 - J51_1, I52 = J52_2 - J52_1;
    double g0 = 2.0*I30 + 3.0*a*a*I50;
    double g1 = 2.0*I31 + 3.0*a*a*I51;

    double c[3], rxb[3], txb[3];
    cross3(b, t, c);
    cross3(rho, b, rxb);
    cross3(t, b, txb);
    double q = dot3(c, rho);
    double k1 = mu / (8.0 * DDO_PI);
    double k2 = mu / (4.0 * DDO_PI * (1.0 - nu));

    double S[3][3] = {{0}};
    sym_add(S, -k1 * g0, rxb, t);
    sym_add(S,  k1 * g1, txb, t);
    for (int i = 0; i < 3; ++i) S[i][i] += k2 * q * (I30 + 3.0*a*a*I50);
    sym_add(S, -k2 * I30, rho, c);
    sym_add(S,  k2 * I31, t, c);
    outer_add(S, 3.0*k2*q*I50, rho, rho);
    sym_add(S, -3.0*k2*q*I51, rho, t);
    outer_add(S, 3.0*k2*q*I52, t, t);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) sig[3*i + j] = S[i][j];
}

/* Brute-force check mode: the same segment stress by n-point Gauss-Legendre   */
/* quadrature of the integrand along the source (n up to DDO_MAX_Q, composite */
/* over n_panels equal panels).                                               */
void ddo_segment_stress_quad(const double x[3], const double x1[3], const double x2[3],
                             const double b[3], double mu, double nu, double a,
                             int n, int n_panels, double sig[9])
{
    double s[DDO_MAX_Q], w[DDO_MAX_Q];
    ddo_gauss_legendre(n, s, w);
    double d[3] = { x2[0]-x1[0], x2[1]-x1[1], x2[2]-x1[2] };
    double L = sqrt(dot3(d, d));
    double t[3] = { d[0]/L, d[1]/L, d[2]/L };
    for (int k = 0; k < 9; ++k) sig[k] = 0.0;
    double h = 1.0 / n_panels;
    for (int p = 0; p < n_panels; ++p)
        for (int g = 0; g < n; ++g) {
            double sp = (p + s[g]) * h;
            double R[3] = { x[0] - x1[0] - sp*d[0], x[1] - x1[1] - sp*d[1], x[2] - x1[2] - sp*d[2] };
            double K[9];
            ddo_kernel(R, b, t, mu, nu, a, K);
            for (int k = 0; k < 9; ++k) sig[k] += w[g] * h * L * K[k];
        }
}

/* ------------------------------------------------------------------------- */
/* Exact target integral of one pair.  Target segment xa -> xb (length Lt,   */
/* unit tangent t, Burgers vector bj), source segment y1 -> y2 (Burgers bi). */
/* What the source sends to the target's two nodes is                       */
/*   F1 = Lt int_0^1 (1 - u) f(u) du,   F2 = Lt int_0^1 u f(u) du,           */
/*   f(u) = (sigma^i(xa + u (xb - xa)) bj) x t                               */
/* (the Peach-Koehler force of Sec. 2.1 against the linear shape functions), */
/* i.e. the Q-point rule of the nodal-force routine with Q -> infinity.      */
/* Computed by globally adaptive bisection: each panel carries its 10-point  */
/* Gauss-Legendre value and the sum over its two halves; the difference of  */
/* the two is its error estimate and the sum its value.  The panel with the  */
/* largest estimate is split until the estimates add up to at most 1e-14     */
/* times the largest integrand component seen on a 65-point sample of        */
/* [0, 1], or 2048 panels are reached (only the integrand's own rounding     */
/* noise, a few 1e-15 of its scale or 1e-13 for a target on the source's own  */
/* line, keeps the estimates from shrinking further).                        */
/* ------------------------------------------------------------------------- */
#define DDO_EXACT_N 10

typedef struct {
    double xa[3], d[3], t[3], bj[3], Lt;
    double y1[3], y2[3], bi[3];
    double mu, nu, a;
    double s[DDO_EXACT_N], w[DDO_EXACT_N];
} ddo_pair_ctx;

/* out[0..2] = (1 - u) f(u), out[3..5] = u f(u) */
static void pair_integrand(const ddo_pair_ctx *P, double u, double out[6])
{
    double xq[3] = { P->xa[0] + u*P->d[0], P->xa[1] + u*P->d[1], P->xa[2] + u*P->d[2] };
    double sg[9], sb[3], f[3];
    ddo_segment_stress(xq, P->y1, P->y2, P->bi, P->mu, P->nu, P->a, sg);
    for (int r = 0; r < 3; ++r) sb[r] = sg[3*r]*P->bj[0] + sg[3*r + 1]*P->bj[1] + sg[3*r + 2]*P->bj[2];
    cross3(sb, P->t, f);
    for (int r = 0; r < 3; ++r) {
        out[r] = (1.0 - u) * f[r];
        out[3 + r] = u * f[r];
    }
}

static void pair_panel(const ddo_pair_ctx *P, double lo, double hi, double out[6])
{
    for (int k = 0; k < 6; ++k) out[k] = 0.0;
    for (int g = 0; g < DDO_EXACT_N; ++g) {
        double v[6];
        pair_integrand(P, lo + P->s[g] * (hi - lo), v);
        for (int k = 0; k < 6; ++k) out[k] += P->w[g] * (hi - lo) * v[k];
    }
}

#define DDO_EXACT_MAXP 2048

typedef struct { double lo, hi, whole[6], value[6], err; } ddo_panel;

/* fills value and err of a panel whose lo, hi and whole are set */
static void pair_refine(const ddo_pair_ctx *P, ddo_panel *q)
{
    double mid = 0.5 * (q->lo + q->hi), left[6], right[6];
    pair_panel(P, q->lo, mid, left);
    pair_panel(P, mid, q->hi, right);
    q->err = 0.0;
    for (int k = 0; k < 6; ++k) {
        q->value[k] = left[k] + right[k];
        q->err = fmax(q->err, fabs(q->value[k] - q->whole[k]));
    }
}

int ddo_pair_exact(const double xa[3], const double xb[3], const double bj[3],
                   const double y1[3], const double y2[3], const double bi[3],
                   double mu, double nu, double a, double F1[3], double F2[3])
{
    ddo_pair_ctx P;
    for (int r = 0; r < 3; ++r) {
        P.xa[r] = xa[r];
        P.d[r] = xb[r] - xa[r];
        P.bj[r] = bj[r];
        P.y1[r] = y1[r];
        P.y2[r] = y2[r];
        P.bi[r] = bi[r];
    }
    P.Lt = sqrt(dot3(P.d, P.d));
    if (!(P.Lt > 0.0)) return -1;
    for (int r = 0; r < 3; ++r) P.t[r] = P.d[r] / P.Lt;
    P.mu = mu; P.nu = nu; P.a = a;
    ddo_gauss_legendre(DDO_EXACT_N, P.s, P.w);
    double scale = 0.0;
    for (int k = 0; k <= 64; ++k) {
        double v[6];
        pair_integrand(&P, k / 64.0, v);
        for (int c = 0; c < 6; ++c) scale = fmax(scale, fabs(v[c]));
    }
    double acc[6] = {0};
    if (scale > 0.0) {
        ddo_panel *pan = (ddo_panel *)malloc(sizeof(ddo_panel) * DDO_EXACT_MAXP);
        if (!pan) return -1;
        int np = 1;
        pan[0].lo = 0.0;
        pan[0].hi = 1.0;
        pair_panel(&P, 0.0, 1.0, pan[0].whole);
        pair_refine(&P, &pan[0]);
        for (;;) {
            double total = 0.0;
            int worst = 0;
            for (int k = 0; k < np; ++k) {
                total += pan[k].err;
                if (pan[k].err > pan[worst].err) worst = k;
            }
            if (total <= 1e-14 * scale || np + 1 > DDO_EXACT_MAXP) break;
            /* split the worst panel: its halves become panels of their own */
            ddo_panel *q = &pan[worst], *r = &pan[np++];
            double mid = 0.5 * (q->lo + q->hi);
            r->lo = mid;
            r->hi = q->hi;
            pair_panel(&P, mid, q->hi, r->whole);
            q->hi = mid;
            pair_panel(&P, q->lo, mid, q->whole);
            pair_refine(&P, q);
            pair_refine(&P, r);
        }
        for (int k = 0; k < np; ++k)
            for (int c = 0; c < 6; ++c) acc[c] += pan[k].value[c];
        free(pan);
    }
    for (int r = 0; r < 3; ++r) {
        F1[r] = P.Lt * acc[r];
        F2[r] = P.Lt * acc[3 + r];
    }
    return 0;
}

/* The exact band: a pair (target j, source i) is near when                  */
/*   |S_i - S_j|^2 < 2 eta^2 (|D_i|^2 + |D_j|^2),                            */
/* S = x1 + x2 (twice the midpoint), D = x2 - x1, i.e. when the midpoints are */
/* closer than eta sqrt((L_i^2 + L_j^2)/2).  Near pairs take the exact       */
/* target integral above, all others the Q-point rule.  eta = 0 (the         */
/* default) takes the Q-point rule everywhere.  The products and sums are    */
/* written out in this order so that the decision is reproducible exactly.  */
static double g_exact_c2 = 0.0;   /* 2 eta^2 */

int ddo_set_exact_band(double eta)
{
    if (!(eta >= 0.0) || isinf(eta)) return -1;
    g_exact_c2 = 2.0 * eta * eta;
    return 0;
}

static int near_pair(const double *xa, const double *xb, const double *y1, const double *y2)
{
    if (!(g_exact_c2 > 0.0)) return 0;
    double e0 = (y1[0] + y2[0]) - (xa[0] + xb[0]);
    double e1 = (y1[1] + y2[1]) - (xa[1] + xb[1]);
    double e2 = (y1[2] + y2[2]) - (xa[2] + xb[2]);
    double di0 = y2[0] - y1[0], di1 = y2[1] - y1[1], di2 = y2[2] - y1[2];
    double dj0 = xb[0] - xa[0], dj1 = xb[1] - xa[1], dj2 = xb[2] - xa[2];
    double dd = e0*e0 + e1*e1 + e2*e2;
    double Di = di0*di0 + di1*di1 + di2*di2;
    double Dj = dj0*dj0 + dj1*dj1 + dj2*dj2;
    return dd < g_exact_c2 * (Di + Dj);
}

/* ------------------------------------------------------------------------- */
/* Nodal forces: for every target segment j and Gauss point q,               */
/*   sigma(x_jq) = sigma_app + sum_{i != j} sigma^i(x_jq)  (sources in order) */
/*   f_jq = (sigma b_j) x t_j                      (Peach-Koehler, Sec. 2.1) */
/*   F[n1(j)] += L_j w_q (1 - s_q) f_jq,  F[n2(j)] += L_j w_q s_q f_jq       */
/* include_self = 1 also adds the segment's own field (a variant).          */
/* ------------------------------------------------------------------------- */
/* Source field used by the force routines: the closed form (default), or,  */
/* after ddo_set_source_quadrature(n, panels) with n > 0, n-point            */
/* Gauss-Legendre quadrature of the integrand on `panels` equal panels of    */
/* the source (ddo_segment_stress_quad).  The quadrature is the slow         */
/* reference where the closed form's endpoint differences lose digits (a    */
/* screw source seen from far along its own axis).                          */
static int g_srcq_n = 0, g_srcq_panels = 0;

int ddo_set_source_quadrature(int n, int panels)
{
    if (n < 0 || n > DDO_MAX_Q || (n > 0 && panels < 1)) return -1;
    g_srcq_n = n;
    g_srcq_panels = panels;
    return 0;
}

static void source_stress(const double xq[3], const double y1[3], const double y2[3], const double bi[3],
                          const ddo_material *m, double sg[9])
{
    if (g_srcq_n > 0)
        ddo_segment_stress_quad(xq, y1, y2, bi, m->mu, m->nu, m->a, g_srcq_n, g_srcq_panels, sg);
    else
        ddo_segment_stress(xq, y1, y2, bi, m->mu, m->nu, m->a, sg);
}

/* What target segment j sends to its two nodes: out[0..2] to node 1 and     */
/* out[3..5] to node 2, Gauss points in order, each point's contributions    */
/* added in the order (w1 f to node 1, w2 f to node 2); then the exact band. */
static int target_end_forces(int64_t n_nodes, const double *x, int64_t n_segs,
                             const int32_t *seg_nodes, const double *burgers,
                             double Sapp[3][3], const ddo_material *m, int n_gauss,
                             const double *s, const double *w, int include_self, int64_t j,
                             double *out, double near_out[6])
{
    const double *X = x, *Y = x + n_nodes, *Z = x + 2*n_nodes;
    const int32_t *N1 = seg_nodes, *N2 = seg_nodes + n_segs;
    int32_t a1 = N1[j], a2 = N2[j];
    double xa[3] = { X[a1], Y[a1], Z[a1] }, xb[3] = { X[a2], Y[a2], Z[a2] };
    double d[3] = { xb[0]-xa[0], xb[1]-xa[1], xb[2]-xa[2] };
    double L = sqrt(dot3(d, d));
    if (!(L > 0.0)) return -1;
    double t[3] = { d[0]/L, d[1]/L, d[2]/L };
    double bj[3] = { burgers[j], burgers[n_segs + j], burgers[2*n_segs + j] };
    for (int g = 0; g < n_gauss; ++g) {
        double xq[3] = { xa[0] + s[g]*d[0], xa[1] + s[g]*d[1], xa[2] + s[g]*d[2] };
        double S[3][3];
        memcpy(S, Sapp, sizeof S);
        for (int64_t i = 0; i < n_segs; ++i) {
            if (i == j && !include_self) continue;
            int32_t c1 = N1[i], c2 = N2[i];
            double y1[3] = { X[c1], Y[c1], Z[c1] }, y2[3] = { X[c2], Y[c2], Z[c2] };
            if (near_pair(xa, xb, y1, y2)) continue;
            double bi[3] = { burgers[i], burgers[n_segs + i], burgers[2*n_segs + i] };
            double sg[9];
            source_stress(xq, y1, y2, bi, m, sg);
            for (int r = 0; r < 3; ++r)
                for (int cc = 0; cc < 3; ++cc) S[r][cc] += sg[3*r + cc];
        }
        double sb[3], f[3];
        for (int r = 0; r < 3; ++r) sb[r] = S[r][0]*bj[0] + S[r][1]*bj[1] + S[r][2]*bj[2];
        cross3(sb, t, f);
        double w1 = L * w[g] * (1.0 - s[g]), w2 = L * w[g] * s[g];
        for (int r = 0; r < 3; ++r) {
            out[6*g + r] = w1 * f[r];
            out[6*g + 3 + r] = w2 * f[r];
        }
    }
    /* near pairs: the exact target integral, summed over sources in order */
    for (int k = 0; k < 6; ++k) near_out[k] = 0.0;
    for (int64_t i = 0; i < n_segs && g_exact_c2 > 0.0; ++i) {
        if (i == j && !include_self) continue;
        int32_t c1 = N1[i], c2 = N2[i];
        double y1[3] = { X[c1], Y[c1], Z[c1] }, y2[3] = { X[c2], Y[c2], Z[c2] };
        if (!near_pair(xa, xb, y1, y2)) continue;
        double bi[3] = { burgers[i], burgers[n_segs + i], burgers[2*n_segs + i] };
        double F1[3], F2[3];
        if (ddo_pair_exact(xa, xb, bj, y1, y2, bi, m->mu, m->nu, m->a, F1, F2)) return -1;
        for (int r = 0; r < 3; ++r) {
            near_out[r] += F1[r];
            near_out[3 + r] += F2[r];
        }
    }
    return 0;
}

/* Targets are independent: each computes its own end forces (in parallel   */
/* when this file is compiled with OpenMP, for the CPU baseline's            */
/* multi-core leg; the plain build ignores the pragma), then they are added  */
/* to the nodes in target order, which gives the same sums, bit for bit, as  */
/* one thread adding each contribution as it is computed.  Near-pair         */
/* contributions are added after the target's Gauss points.                  */
static int ddo_forces_impl(int64_t n_nodes, const double *x, int64_t n_segs,
                           const int32_t *seg_nodes, const double *burgers,
                           const double sigma_app[6], const ddo_material *m,
                           int n_gauss, int include_self,
                           int64_t tgt_begin, int64_t tgt_end, double *force_out)
{
    double s[DDO_MAX_Q], w[DDO_MAX_Q];
    if (ddo_gauss_legendre(n_gauss, s, w)) return -1;
    const int32_t *N1 = seg_nodes, *N2 = seg_nodes + n_segs;
    for (int64_t k = 0; k < 3*n_nodes; ++k) force_out[k] = 0.0;
    double Sapp[3][3];
    voigt_to_full(sigma_app, Sapp);
    int64_t nt = tgt_end - tgt_begin;
    if (nt <= 0) return 0;
    double *ends = malloc(sizeof(double) * 6 * (size_t)n_gauss * (size_t)nt);
    double (*nears)[6] = malloc(sizeof(*nears) * (size_t)nt);
    if (!ends || !nears) {
        free(ends);
        free(nears);
        return -1;
    }
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(| : bad)
    for (int64_t j = tgt_begin; j < tgt_end; ++j)
        bad |= target_end_forces(n_nodes, x, n_segs, seg_nodes, burgers, Sapp, m, n_gauss, s, w,
                                 include_self, j, ends + 6 * n_gauss * (j - tgt_begin), nears[j - tgt_begin]) != 0;
    for (int64_t j = tgt_begin; j < tgt_end && !bad; ++j) {
        int32_t a1 = N1[j], a2 = N2[j];
        const double *e = ends + 6 * n_gauss * (j - tgt_begin);
        for (int g = 0; g < n_gauss; ++g)
            for (int r = 0; r < 3; ++r) {
                force_out[r*n_nodes + a1] += e[6*g + r];
                force_out[r*n_nodes + a2] += e[6*g + 3 + r];
            }
        if (g_exact_c2 > 0.0)
            for (int r = 0; r < 3; ++r) {
                force_out[r*n_nodes + a1] += nears[j - tgt_begin][r];
                force_out[r*n_nodes + a2] += nears[j - tgt_begin][3 + r];
            }
    }
    free(ends);
    free(nears);
    return bad ? -1 : 0;
}

/* Number of threads the force routines use (1 for the plain build). */
int ddo_threads(void)
{
#ifdef _OPENMP
    int n = 1;
#pragma omp parallel
#pragma omp master
    n = omp_get_num_threads();
    return n;
#else
    return 1;
#endif
}

static int check_topology(int64_t n_nodes, int64_t n_segs, const int32_t *seg_nodes)
{
    for (int64_t k = 0; k < 2*n_segs; ++k)
        if (seg_nodes[k] < 0 || seg_nodes[k] >= n_nodes) return -1;
    return 0;
}

int ddo_nodal_forces(int64_t n_nodes, const double *x, int64_t n_segs,
                     const int32_t *seg_nodes, const double *burgers,
                     const double *normal, const double sigma_app[6],
                     const ddo_material *m, int n_gauss, int include_self,
                     double *force_out)
{
    (void)normal;
    if (n_nodes < 0 || n_segs < 0 || !m || n_gauss < 1 || n_gauss > DDO_MAX_Q) return -1;
    if (check_topology(n_nodes, n_segs, seg_nodes)) return -1;
    return ddo_forces_impl(n_nodes, x, n_segs, seg_nodes, burgers, sigma_app, m,
                           n_gauss, include_self, 0, n_segs, force_out);
}

/* Forces from the Gauss points of target segments [tgt_begin, tgt_end) only, */
/* against all sources (sampled checks of large volumes).  Nodes touched by   */
/* no sampled segment stay 0.                                                 */
int ddo_nodal_forces_sampled(int64_t n_nodes, const double *x, int64_t n_segs,
                             const int32_t *seg_nodes, const double *burgers,
                             const double sigma_app[6], const ddo_material *m,
                             int n_gauss, int64_t tgt_begin, int64_t tgt_end,
                             double *force_out)
{
    if (tgt_begin < 0 || tgt_end > n_segs || tgt_begin > tgt_end) return -1;
    if (check_topology(n_nodes, n_segs, seg_nodes)) return -1;
    return ddo_forces_impl(n_nodes, x, n_segs, seg_nodes, burgers, sigma_app, m,
                           n_gauss, 0, tgt_begin, tgt_end, force_out);
}

/* Per-segment end forces: out[6*j + 0..2] is what segment j sends to its     */
/* node 1, out[6*j + 3..5] to its node 2 (same quadrature as above), for j in */
/* [tgt_begin, tgt_end).                                                      */
int ddo_segment_end_forces(int64_t n_nodes, const double *x, int64_t n_segs,
                           const int32_t *seg_nodes, const double *burgers,
                           const double sigma_app[6], const ddo_material *m,
                           int n_gauss, int64_t tgt_begin, int64_t tgt_end,
                           double *out)
{
    double s[DDO_MAX_Q], w[DDO_MAX_Q];
    if (ddo_gauss_legendre(n_gauss, s, w)) return -1;
    if (check_topology(n_nodes, n_segs, seg_nodes)) return -1;
    const double *X = x, *Y = x + n_nodes, *Z = x + 2*n_nodes;
    const int32_t *N1 = seg_nodes, *N2 = seg_nodes + n_segs;
    double Sapp[3][3];
    voigt_to_full(sigma_app, Sapp);
    for (int64_t j = tgt_begin; j < tgt_end; ++j) {
        double *o = out + 6*(j - tgt_begin);
        for (int k = 0; k < 6; ++k) o[k] = 0.0;
        int32_t a1 = N1[j], a2 = N2[j];
        double xa[3] = { X[a1], Y[a1], Z[a1] }, xb[3] = { X[a2], Y[a2], Z[a2] };
        double d[3] = { xb[0]-xa[0], xb[1]-xa[1], xb[2]-xa[2] };
        double L = sqrt(dot3(d, d));
        double t[3] = { d[0]/L, d[1]/L, d[2]/L };
        double bj[3] = { burgers[j], burgers[n_segs + j], burgers[2*n_segs + j] };
        for (int g = 0; g < n_gauss; ++g) {
            double xq[3] = { xa[0] + s[g]*d[0], xa[1] + s[g]*d[1], xa[2] + s[g]*d[2] };
            double S[3][3];
            memcpy(S, Sapp, sizeof S);
            for (int64_t i = 0; i < n_segs; ++i) {
                if (i == j) continue;
                int32_t c1 = N1[i], c2 = N2[i];
                double y1[3] = { X[c1], Y[c1], Z[c1] }, y2[3] = { X[c2], Y[c2], Z[c2] };
                if (near_pair(xa, xb, y1, y2)) continue;
                double bi[3] = { burgers[i], burgers[n_segs + i], burgers[2*n_segs + i] };
                double sg[9];
                ddo_segment_stress(xq, y1, y2, bi, m->mu, m->nu, m->a, sg);
                for (int r = 0; r < 3; ++r)
                    for (int cc = 0; cc < 3; ++cc) S[r][cc] += sg[3*r + cc];
            }
            double sb[3], f[3];
            for (int r = 0; r < 3; ++r) sb[r] = S[r][0]*bj[0] + S[r][1]*bj[1] + S[r][2]*bj[2];
            cross3(sb, t, f);
            for (int r = 0; r < 3; ++r) {
                o[r]     += L * w[g] * (1.0 - s[g]) * f[r];
                o[3 + r] += L * w[g] * s[g] * f[r];
            }
        }
        for (int64_t i = 0; i < n_segs && g_exact_c2 > 0.0; ++i) {
            if (i == j) continue;
            int32_t c1 = N1[i], c2 = N2[i];
            double y1[3] = { X[c1], Y[c1], Z[c1] }, y2[3] = { X[c2], Y[c2], Z[c2] };
            if (!near_pair(xa, xb, y1, y2)) continue;
            double bi[3] = { burgers[i], burgers[n_segs + i], burgers[2*n_segs + i] };
            double F1[3], F2[3];
            if (ddo_pair_exact(xa, xb, bj, y1, y2, bi, m->mu, m->nu, m->a, F1, F2)) return -1;
            for (int r = 0; r < 3; ++r) {
                o[r] += F1[r];
                o[3 + r] += F2[r];
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Glide mobility, lumped form of Eq. DD_evol with scalar drag B:            */
/*   ell_n = 1/2 sum_{s attached to n} L_s                                   */
/*   v_n   = P_n F_n / (B ell_n)                                             */
/* P_n removes the climb component: with one distinct slip-plane normal     */
/* among the attached segments, P = I - n n^T; with two, v is projected on   */
/* their intersection line n1 x n2; with three or more, v = 0.  Pinned or    */
/* unattached nodes get v = 0.  Then x_n += v_n dt (forward Euler).          */
/* ------------------------------------------------------------------------- */
static void node_velocities(int64_t n_nodes, const double *x, const double *force,
                            int64_t n_segs, const int32_t *seg_nodes,
                            const double *normal, const uint8_t *pinned,
                            const ddo_material *m, double *vel)
{
    const int32_t *N1 = seg_nodes, *N2 = seg_nodes + n_segs;
    double *ell = (double *)calloc((size_t)(n_nodes > 0 ? n_nodes : 1), sizeof(double));
    /* distinct normals per node: up to 3 kept */
    double *nrm = (double *)calloc((size_t)(n_nodes > 0 ? n_nodes : 1) * 9, sizeof(double));
    int *cnt = (int *)calloc((size_t)(n_nodes > 0 ? n_nodes : 1), sizeof(int));
    for (int64_t s = 0; s < n_segs; ++s) {
        int32_t ends[2] = { N1[s], N2[s] };
        double d[3];
        for (int r = 0; r < 3; ++r) d[r] = x[r*n_nodes + ends[1]] - x[r*n_nodes + ends[0]];
        double L = sqrt(dot3(d, d));
        double ns[3] = { normal[s], normal[n_segs + s], normal[2*n_segs + s] };
        for (int e = 0; e < 2; ++e) {
            int64_t n = ends[e];
            ell[n] += 0.5 * L;
            int dup = 0;
            for (int k = 0; k < cnt[n] && k < 3; ++k)
                if (fabs(dot3(&nrm[9*n + 3*k], ns)) > 1.0 - 1e-12) dup = 1;
            if (!dup) {
                if (cnt[n] < 3) memcpy(&nrm[9*n + 3*cnt[n]], ns, sizeof ns);
                cnt[n] += 1;
            }
        }
    }
    for (int64_t n = 0; n < n_nodes; ++n) {
        double F[3] = { force[n], force[n_nodes + n], force[2*n_nodes + n] };
        double v[3] = { 0.0, 0.0, 0.0 };
        if (!(pinned && pinned[n]) && ell[n] > 0.0 && cnt[n] > 0 && cnt[n] < 3) {
            for (int r = 0; r < 3; ++r) v[r] = F[r] / (m->B * ell[n]);
            if (cnt[n] == 1) {
                const double *nn = &nrm[9*n];
                double vn = dot3(v, nn);
                for (int r = 0; r < 3; ++r) v[r] -= vn * nn[r];
            } else {
                double l[3];
                cross3(&nrm[9*n], &nrm[9*n + 3], l);
                double ll = sqrt(dot3(l, l));
                for (int r = 0; r < 3; ++r) l[r] /= ll;
                double vl = dot3(v, l);
                for (int r = 0; r < 3; ++r) v[r] = vl * l[r];
            }
        }
        for (int r = 0; r < 3; ++r) vel[r*n_nodes + n] = v[r];
    }
    free(ell); free(nrm); free(cnt);
}

int ddo_glide_step(int64_t n_nodes, double *x, const double *force, int64_t n_segs,
                   const int32_t *seg_nodes, const double *normal,
                   const uint8_t *pinned, const ddo_material *m, double dt,
                   double *vel_out)
{
    if (n_nodes < 0 || n_segs < 0 || !m || !(m->B > 0.0) || !(dt > 0.0)) return -1;
    if (check_topology(n_nodes, n_segs, seg_nodes)) return -1;
    double *v = (double *)malloc(sizeof(double) * (size_t)(3 * (n_nodes > 0 ? n_nodes : 1)));
    node_velocities(n_nodes, x, force, n_segs, seg_nodes, normal, pinned, m, v);
    for (int64_t k = 0; k < 3*n_nodes; ++k) x[k] += v[k] * dt;
    if (vel_out) memcpy(vel_out, v, sizeof(double) * (size_t)(3*n_nodes));
    free(v);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* FCC slip systems: plane normals (1,1,1), (-1,1,1), (1,-1,1), (1,1,-1)     */
/* over sqrt(3); in each plane the three <110> directions normal to it, the  */
/* one with zero x first, then zero y, then zero z, first non-zero entry     */
/* positive, over sqrt(2).  System alpha = 3 p + d.                          */
/* ------------------------------------------------------------------------- */
static void fcc_system(int alpha, double n[3], double mdir[3])
{
    static const double P[4][3] = { {1,1,1}, {-1,1,1}, {1,-1,1}, {1,1,-1} };
    int p = alpha / 3, d = alpha % 3;
    double r3 = 1.0 / sqrt(3.0), r2 = 1.0 / sqrt(2.0);
    for (int k = 0; k < 3; ++k) n[k] = P[p][k] * r3;
    /* direction with component d equal to zero, perpendicular to n */
    int i1 = (d + 1) % 3, i2 = (d + 2) % 3;
    double v[3] = { 0, 0, 0 };
    /* need v[i1]*P[i1] + v[i2]*P[i2] = 0 with |v[i1]| = |v[i2]| = 1 */
    v[i1] = 1.0;
    v[i2] = -P[p][i1] / P[p][i2];
    /* make the first non-zero entry positive */
    int first = (v[0] != 0.0) ? 0 : (v[1] != 0.0 ? 1 : 2);
    double sgn = v[first] > 0 ? 1.0 : -1.0;
    for (int k = 0; k < 3; ++k) mdir[k] = sgn * v[k] * r2;
}

void ddo_fcc_system(int alpha, double n[3], double m[3]) { fcc_system(alpha, n, m); }

/* System of a segment: the alpha whose plane normal matches n_s up to sign  */
/* and whose direction matches b_s/|b_s| up to sign; -1 if none.             */
static int segment_system(const double ns[3], const double bs[3])
{
    double bl = sqrt(dot3(bs, bs));
    if (!(bl > 0.0)) return -1;
    for (int al = 0; al < 12; ++al) {
        double n[3], md[3];
        fcc_system(al, n, md);
        if (fabs(dot3(n, ns)) > 1.0 - 1e-6 && fabs(dot3(md, bs)) / bl > 1.0 - 1e-6) return al;
    }
    return -1;
}

/* Resolved shear stress tau_alpha = m_alpha . sigma n_alpha (numerator of  */
/* Eq. schmid) for the 12 systems.                                           */
void ddo_resolved_shear(const double sigma[6], double tau[12])
{
    double S[3][3];
    voigt_to_full(sigma, S);
    for (int al = 0; al < 12; ++al) {
        double n[3], md[3], Sn[3];
        fcc_system(al, n, md);
        for (int r = 0; r < 3; ++r) Sn[r] = S[r][0]*n[0] + S[r][1]*n[1] + S[r][2]*n[2];
        tau[al] = dot3(md, Sn);
    }
}

/* Per-system slip rate of one configuration with node velocities v:         */
/*  gdot_alpha = (1/V) sum_{s in alpha} (b_s.m_alpha) L_s ((t_s x vbar_s).n_alpha) */
/* vbar_s = (v_n1 + v_n2)/2.  This is the segment distortion rate             */
/* b/A (x) (l x V) times l A, summed and divided by the volume, resolved on  */
/* (m_alpha, n_alpha).                                                        */
static void slip_rates(int64_t n_nodes, const double *x, const double *vel,
                       int64_t n_segs, const int32_t *seg_nodes, const double *burgers,
                       const double *normal, double volume, double out[12])
{
    const int32_t *N1 = seg_nodes, *N2 = seg_nodes + n_segs;
    for (int al = 0; al < 12; ++al) out[al] = 0.0;
    for (int64_t s = 0; s < n_segs; ++s) {
        double ns[3] = { normal[s], normal[n_segs + s], normal[2*n_segs + s] };
        double bs[3] = { burgers[s], burgers[n_segs + s], burgers[2*n_segs + s] };
        int al = segment_system(ns, bs);
        if (al < 0) continue;
        double n[3], md[3];
        fcc_system(al, n, md);
        int32_t a1 = N1[s], a2 = N2[s];
        double d[3], vb[3];
        for (int r = 0; r < 3; ++r) {
            d[r] = x[r*n_nodes + a2] - x[r*n_nodes + a1];
            vb[r] = 0.5 * (vel[r*n_nodes + a1] + vel[r*n_nodes + a2]);
        }
        double L = sqrt(dot3(d, d));
        double t[3] = { d[0]/L, d[1]/L, d[2]/L }, txv[3];
        cross3(t, vb, txv);
        out[al] += dot3(bs, md) * L * dot3(txv, n) / volume;
    }
}

/* Per-system mobile and sessile densities (line length per volume).  A     */
/* segment is sessile when both of its nodes are pinned.                     */
static void densities(int64_t n_nodes, const double *x, int64_t n_segs,
                      const int32_t *seg_nodes, const double *burgers,
                      const double *normal, const uint8_t *pinned, double volume,
                      double mob[12], double ses[12])
{
    const int32_t *N1 = seg_nodes, *N2 = seg_nodes + n_segs;
    for (int al = 0; al < 12; ++al) mob[al] = ses[al] = 0.0;
    for (int64_t s = 0; s < n_segs; ++s) {
        double ns[3] = { normal[s], normal[n_segs + s], normal[2*n_segs + s] };
        double bs[3] = { burgers[s], burgers[n_segs + s], burgers[2*n_segs + s] };
        int al = segment_system(ns, bs);
        if (al < 0) continue;
        int32_t a1 = N1[s], a2 = N2[s];
        double d[3];
        for (int r = 0; r < 3; ++r) d[r] = x[r*n_nodes + a2] - x[r*n_nodes + a1];
        double L = sqrt(dot3(d, d));
        int sessile = pinned && pinned[a1] && pinned[a2];
        if (sessile) ses[al] += L / volume; else mob[al] += L / volume;
    }
}

/* ------------------------------------------------------------------------- */
/* One burst at frozen load (the fast equation, Eq. fast_dd, at fixed       */
/* applied stress): n_steps forward-Euler glide steps.  At step k the forces */
/* and velocities of X_k give gdot(k); R = (1/K) sum_k gdot(k) is the running */
/* time average with equal steps (Eq. R_lambda_t).  features_out (nullable): */
/* [0..11] tau_alpha, [12..23] mobile density, [24..35] sessile density, of  */
/* the initial state.  x is advanced in place.                               */
/* ------------------------------------------------------------------------- */
int ddo_burst(int64_t n_nodes, double *x, int64_t n_segs, const int32_t *seg_nodes,
              const double *burgers, const double *normal, const uint8_t *pinned,
              const double sigma_app[6], double volume, const ddo_material *m,
              int n_gauss, int n_steps, double dt, double rate_avg_out[12],
              double *features_out)
{
    if (n_steps < 0 || !(dt > 0.0) || !(volume > 0.0)) return -1;
    if (check_topology(n_nodes, n_segs, seg_nodes)) return -1;
    size_t nn = (size_t)(3 * (n_nodes > 0 ? n_nodes : 1));
    double *F = (double *)malloc(sizeof(double) * nn);
    double *v = (double *)malloc(sizeof(double) * nn);
    if (features_out) {
        ddo_resolved_shear(sigma_app, features_out);
        densities(n_nodes, x, n_segs, seg_nodes, burgers, normal, pinned, volume,
                  features_out + 12, features_out + 24);
    }
    double acc[12] = {0};
    for (int k = 0; k < n_steps; ++k) {
        if (ddo_forces_impl(n_nodes, x, n_segs, seg_nodes, burgers, sigma_app, m,
                            n_gauss, 0, 0, n_segs, F)) { free(F); free(v); return -1; }
        node_velocities(n_nodes, x, F, n_segs, seg_nodes, normal, pinned, m, v);
        double g[12];
        slip_rates(n_nodes, x, v, n_segs, seg_nodes, burgers, normal, volume, g);
        for (int al = 0; al < 12; ++al) acc[al] += g[al];
        for (size_t i = 0; i < (size_t)(3*n_nodes); ++i) x[i] += v[i] * dt;
    }
    for (int al = 0; al < 12; ++al) rate_avg_out[al] = n_steps > 0 ? acc[al] / n_steps : 0.0;
    free(F); free(v);
    return 0;
}

/* Independent bursts, one after another: instance i owns nodes              */
/* [node_off[i], node_off[i+1]) and segments [seg_off[i], seg_off[i+1]);     */
/* seg_nodes are instance-local.                                             */
int ddo_burst_batch(int32_t n_inst, const int64_t *node_off, const int64_t *seg_off,
                    double *x, const int32_t *seg_nodes, const double *burgers,
                    const double *normal, const uint8_t *pinned,
                    const double *sigma_app, const double *volume,
                    const ddo_material *m, int n_gauss, int n_steps, double dt,
                    double *rate_avg_out, double *features_out)
{
    int64_t NN = node_off[n_inst], NS = seg_off[n_inst];
    for (int32_t i = 0; i < n_inst; ++i) {
        int64_t n0 = node_off[i], nn = node_off[i + 1] - n0;
        int64_t s0 = seg_off[i], ns = seg_off[i + 1] - s0;
        double *xi = (double *)malloc(sizeof(double) * (size_t)(3 * (nn > 0 ? nn : 1)));
        int32_t *sn = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * (ns > 0 ? ns : 1)));
        double *bi = (double *)malloc(sizeof(double) * (size_t)(3 * (ns > 0 ? ns : 1)));
        double *ni = (double *)malloc(sizeof(double) * (size_t)(3 * (ns > 0 ? ns : 1)));
        for (int r = 0; r < 3; ++r)
            for (int64_t k = 0; k < nn; ++k) xi[r*nn + k] = x[r*NN + n0 + k];
        for (int r = 0; r < 2; ++r)
            for (int64_t k = 0; k < ns; ++k) sn[r*ns + k] = seg_nodes[r*NS + s0 + k];
        for (int r = 0; r < 3; ++r)
            for (int64_t k = 0; k < ns; ++k) {
                bi[r*ns + k] = burgers[r*NS + s0 + k];
                ni[r*ns + k] = normal[r*NS + s0 + k];
            }
        int rc = ddo_burst(nn, xi, ns, sn, bi, ni, pinned ? pinned + n0 : NULL,
                           sigma_app + 6*i, volume[i], m, n_gauss, n_steps, dt,
                           rate_avg_out + 12*i, features_out ? features_out + 36*i : NULL);
        for (int r = 0; r < 3; ++r)
            for (int64_t k = 0; k < nn; ++k) x[r*NN + n0 + k] = xi[r*nn + k];
        free(xi); free(sn); free(bi); free(ni);
        if (rc) return rc;
    }
    return 0;
}
