/* Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the
 * oracle (oracle/ddo.c): every routine on small inputs held in heap arrays of
 * exactly the documented sizes, including the exact band, the brute-force
 * source quadrature, batches with an empty instance and rejected arguments.
 * Exit status 0 and no sanitizer report = pass.  Test infrastructure only. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct { double mu, nu, a, B; } ddo_material;
int ddo_gauss_legendre(int n, double *s, double *w);
void ddo_kernel(const double R[3], const double b[3], const double t[3], double mu, double nu, double a,
                double out[9]);
void ddo_segment_stress(const double x[3], const double x1[3], const double x2[3], const double b[3], double mu,
                        double nu, double a, double sig[9]);
void ddo_segment_stress_quad(const double x[3], const double x1[3], const double x2[3], const double b[3],
                             double mu, double nu, double a, int n, int n_panels, double sig[9]);
int ddo_pair_exact(const double xa[3], const double xb[3], const double bj[3], const double y1[3],
                   const double y2[3], const double bi[3], double mu, double nu, double a, double F1[3],
                   double F2[3]);
int ddo_set_exact_band(double eta);
int ddo_set_source_quadrature(int n, int panels);
int ddo_nodal_forces(int64_t n_nodes, const double *x, int64_t n_segs, const int32_t *seg_nodes,
                     const double *burgers, const double *normal, const double sigma_app[6],
                     const ddo_material *m, int n_gauss, int include_self, double *force_out);
int ddo_nodal_forces_sampled(int64_t n_nodes, const double *x, int64_t n_segs, const int32_t *seg_nodes,
                             const double *burgers, const double sigma_app[6], const ddo_material *m,
                             int n_gauss, int64_t tgt_begin, int64_t tgt_end, double *force_out);
int ddo_segment_end_forces(int64_t n_nodes, const double *x, int64_t n_segs, const int32_t *seg_nodes,
                           const double *burgers, const double sigma_app[6], const ddo_material *m,
                           int n_gauss, int64_t tgt_begin, int64_t tgt_end, double *out);
int ddo_glide_step(int64_t n_nodes, double *x, const double *force, int64_t n_segs, const int32_t *seg_nodes,
                   const double *normal, const uint8_t *pinned, const ddo_material *m, double dt,
                   double *vel_out);
void ddo_fcc_system(int alpha, double n[3], double m[3]);
void ddo_resolved_shear(const double sigma[6], double tau[12]);
int ddo_burst(int64_t n_nodes, double *x, int64_t n_segs, const int32_t *seg_nodes, const double *burgers,
              const double *normal, const uint8_t *pinned, const double sigma_app[6], double volume,
              const ddo_material *m, int n_gauss, int n_steps, double dt, double rate_avg_out[12],
              double *features_out);
int ddo_burst_batch(int32_t n_inst, const int64_t *node_off, const int64_t *seg_off, double *x,
                    const int32_t *seg_nodes, const double *burgers, const double *normal,
                    const uint8_t *pinned, const double *sigma_app, const double *volume,
                    const ddo_material *m, int n_gauss, int n_steps, double dt, double *rate_avg_out,
                    double *features_out);

static void *xalloc(size_t bytes)
{
    void *p = malloc(bytes ? bytes : 1);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

static int failures = 0;
static void expect(int cond, const char *what)
{
    if (!cond) {
        fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

/* k regular n-gons of radius r in the (111) plane, centres along x, Burgers
 * vector along [1 -1 0]/sqrt 2, SoA layouts of the oracle. */
static void loops(int k, int n, double r, double **x, int32_t **sn, double **b, double **nrm)
{
    const int N = k * n;
    *x = xalloc(sizeof(double) * 3 * N);
    *sn = xalloc(sizeof(int32_t) * 2 * N);
    *b = xalloc(sizeof(double) * 3 * N);
    *nrm = xalloc(sizeof(double) * 3 * N);
    const double s3 = 1.0 / sqrt(3.0), s2 = 1.0 / sqrt(2.0);
    const double nv[3] = {s3, s3, s3}, e1[3] = {s2, -s2, 0.0};
    const double e2[3] = {nv[1] * e1[2] - nv[2] * e1[1], nv[2] * e1[0] - nv[0] * e1[2], nv[0] * e1[1] - nv[1] * e1[0]};
    for (int l = 0; l < k; ++l)
        for (int i = 0; i < n; ++i) {
            const int g = l * n + i;
            const double ph = 2.0 * 3.14159265358979323846 * i / n + 0.3 * l;
            for (int c = 0; c < 3; ++c) {
                (*x)[c * N + g] = (c == 0 ? 700.0 * l : 0.0) + r * (cos(ph) * e1[c] + sin(ph) * e2[c]);
                (*b)[c * N + g] = e1[c];
                (*nrm)[c * N + g] = nv[c];
            }
            (*sn)[g] = g;
            (*sn)[N + g] = l * n + (i + 1) % n;
        }
}

int main(void)
{
    const ddo_material mat = {48e9, 0.34, 1.0, 1e-4};
    /* Gauss-Legendre rules of every order */
    for (int n = 1; n <= 64; ++n) {
        double *s = xalloc(sizeof(double) * n), *w = xalloc(sizeof(double) * n), sum = 0.0;
        expect(ddo_gauss_legendre(n, s, w) == 0, "gauss_legendre");
        for (int i = 0; i < n; ++i) sum += w[i];
        expect(fabs(sum - 1.0) < 1e-13, "weights sum to 1");
        free(s);
        free(w);
    }
    /* elementary pieces */
    double R[3] = {3.0, -2.0, 1.0}, bb[3] = {1.0, 0.0, 0.0}, t[3] = {0.0, 0.0, 1.0}, K[9], S1[9], S2[9];
    ddo_kernel(R, bb, t, mat.mu, mat.nu, mat.a, K);
    const double x1[3] = {0, 0, 0}, x2[3] = {0, 0, 10}, xp[3] = {5, 1, 3};
    ddo_segment_stress(xp, x1, x2, bb, mat.mu, mat.nu, mat.a, S1);
    ddo_segment_stress_quad(xp, x1, x2, bb, mat.mu, mat.nu, mat.a, 64, 64, S2);
    for (int k = 0; k < 9; ++k) expect(fabs(S1[k] - S2[k]) <= 1e-10 * (fabs(S2[k]) + mat.mu * 1e-12), "stress");
    double F1[3], F2[3];
    const double xa[3] = {0, 1, 0}, xb[3] = {0, 1, 8};
    expect(ddo_pair_exact(xa, xb, bb, x1, x2, bb, mat.mu, mat.nu, mat.a, F1, F2) == 0, "pair_exact");
    for (int al = 0; al < 12; ++al) {
        double n3[3], m3[3];
        ddo_fcc_system(al, n3, m3);
    }
    const double sig[6] = {1e7, -2e7, 5e7, 3e6, -4e6, 2e6};
    double tau[12];
    ddo_resolved_shear(sig, tau);

    /* a volume of 3 octagon loops: forces, bands, sampled, end forces, glide */
    double *x, *b, *nrm;
    int32_t *sn;
    const int nl = 3, ng = 8, N = nl * ng;
    loops(nl, ng, 120.0, &x, &sn, &b, &nrm);
    double *F = xalloc(sizeof(double) * 3 * N), *Fb = xalloc(sizeof(double) * 3 * N);
    expect(ddo_nodal_forces(N, x, N, sn, b, nrm, sig, &mat, 2, 0, F) == 0, "nodal_forces");
    expect(ddo_nodal_forces(N, x, N, sn, b, nrm, sig, &mat, 3, 1, F) == 0, "nodal_forces include_self");
    expect(ddo_set_exact_band(2.0) == 0, "set_exact_band");
    expect(ddo_nodal_forces(N, x, N, sn, b, nrm, sig, &mat, 2, 0, Fb) == 0, "nodal_forces with band");
    expect(ddo_set_exact_band(0.0) == 0, "band off");
    expect(ddo_set_source_quadrature(16, 8) == 0, "source quadrature on");
    expect(ddo_nodal_forces(N, x, N, sn, b, nrm, sig, &mat, 2, 0, Fb) == 0, "nodal_forces by quadrature");
    expect(ddo_set_source_quadrature(0, 0) == 0, "source quadrature off");
    expect(ddo_set_source_quadrature(65, 1) != 0, "too many quadrature points rejected");
    expect(ddo_nodal_forces_sampled(N, x, N, sn, b, sig, &mat, 2, 8, 16, F) == 0, "sampled");
    expect(ddo_nodal_forces_sampled(N, x, N, sn, b, sig, &mat, 2, 8, N + 1, F) != 0, "sampled range rejected");
    double *ends = xalloc(sizeof(double) * 6 * 5);
    expect(ddo_segment_end_forces(N, x, N, sn, b, sig, &mat, 4, 3, 8, ends) == 0, "end forces");
    uint8_t *pin = xalloc((size_t)N);
    memset(pin, 0, (size_t)N);
    for (int i = 2 * ng; i < N; ++i) pin[i] = 1;
    double *v = xalloc(sizeof(double) * 3 * N);
    expect(ddo_nodal_forces(N, x, N, sn, b, nrm, sig, &mat, 2, 0, F) == 0, "forces for glide");
    expect(ddo_glide_step(N, x, F, N, sn, nrm, pin, &mat, 2e-14, v) == 0, "glide");
    /* rejected arguments must not read out of bounds */
    int32_t *bad = xalloc(sizeof(int32_t) * 2 * N);
    memcpy(bad, sn, sizeof(int32_t) * 2 * N);
    bad[N + 5] = N;
    expect(ddo_nodal_forces(N, x, N, bad, b, nrm, sig, &mat, 2, 0, F) != 0, "bad index rejected");
    expect(ddo_nodal_forces(N, x, N, sn, b, nrm, sig, &mat, 0, 0, F) != 0, "n_gauss 0 rejected");
    /* a burst with features, and a batch with an empty instance */
    double rate[12], feat[36];
    expect(ddo_burst(N, x, N, sn, b, nrm, pin, sig, 1e12, &mat, 2, 5, 2e-14, rate, feat) == 0, "burst");
    const int64_t no[4] = {0, 2 * ng, 2 * ng, N}, so[4] = {0, 2 * ng, 2 * ng, N};
    int32_t *snl = xalloc(sizeof(int32_t) * 2 * N);
    for (int s = 0; s < N; ++s)
        for (int r = 0; r < 2; ++r) snl[r * N + s] = sn[r * N + s] - (s < 2 * ng ? 0 : 2 * ng);
    double *sigs = xalloc(sizeof(double) * 6 * 3), *vol = xalloc(sizeof(double) * 3);
    for (int i = 0; i < 3; ++i) {
        memcpy(sigs + 6 * i, sig, sizeof sig);
        vol[i] = 1e12;
    }
    double *rates = xalloc(sizeof(double) * 12 * 3), *feats = xalloc(sizeof(double) * 36 * 3);
    expect(ddo_burst_batch(3, no, so, x, snl, b, nrm, pin, sigs, vol, &mat, 2, 3, 2e-14, rates, feats) == 0,
           "burst batch");
    for (int k = 0; k < 3 * N; ++k) expect(isfinite(x[k]), "finite positions");
    free(F); free(Fb); free(ends); free(pin); free(v); free(bad); free(snl); free(sigs); free(vol);
    free(rates); free(feats); free(x); free(sn); free(b); free(nrm);
    printf("oracle sanitizer driver: %d failures\n", failures);
    return failures ? 1 : 0;
}
