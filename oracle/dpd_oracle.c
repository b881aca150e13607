/*
 * FP64 reference ("oracle") for the augmented parallel Hammerstein (APH)
 * digital predistorter of Li et al., "Parallel Digital Predistortion Design on
 * Mobile GPU and Embedded Multicore CPU for Mobile Transmitters".
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, obviously-correct
 * statement of what the predistorter computes.  Only the test-suite, the smoke
 * check and the CPU baseline of the benchmark load it; the library's product
 * path never does.  It shares no code, header, table or helper with the GPU
 * library.
 *
 * Arithmetic: IEEE double, no fast-math, built with -ffp-contract=off.
 * Complex numbers are written out as (re, im) pairs so every product is visible.
 *
 * Functions and the passages they follow:
 *   oracle_forward     Eq. (1) of section 2.1 with the basis functions of
 *                      section 2.1 (odd orders, monomial form) and the three
 *                      steps of Algorithm 1 (polynomial, filtering,
 *                      accumulation + c); zero pre-history as in the
 *                      zero-filled element matrix of Eq. (2).
 *   oracle_forward_at  the same, evaluated only at listed output indices.
 *   oracle_backward    gradient of a real loss through Eq. (1), derived with
 *                      Wirtinger calculus (not in the paper; see below).
 *   oracle_ls_normal   the normal equations Psi^H Psi, Psi^H z of the
 *                      least-squares estimate of section 2.2 (Eq. 2 basis).
 *
 * Coefficient vector (section 2.2 stacking): for each main-branch order in the
 * order given, its L taps h_{p,0..L-1}; then for each conjugate-branch order its
 * L taps (written h-bar in the paper, an independent coefficient here); then
 * the LO-leakage constant c.  K = (n_main + n_conj) * L + 1 complex values,
 * stored as 2K doubles (re, im).
 *
 * Readings taken where the paper is ambiguous:
 *   - the tap sum runs k = 0 .. L-1 (L taps), as the coefficient vectors of
 *     section 2.2 have L entries;
 *   - basis is the monomial |x|^(p-1) x (orthogonal-polynomial constants u are
 *     not given);
 *   - samples before x_0 are zero, or the caller's history when given.
 */
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL 1

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following calls (n >= 1); the timing of the CPU baseline at
   one thread uses it. */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

static int check_orders(const int32_t *orders, int32_t n)
{
    if (n < 0) return 0;
    if (n > 0 && !orders) return 0;
    for (int32_t i = 0; i < n; ++i)
        if (orders[i] < 1 || (orders[i] % 2) == 0) return 0;
    return 1;
}

static int check_args(int64_t n, const int32_t *mo, int32_t nm, const int32_t *co, int32_t nc,
                      int32_t L, const double *coeffs)
{
    if (n < 0 || L < 1 || !coeffs) return 0;
    if (!check_orders(mo, nm) || !check_orders(co, nc)) return 0;
    return 1;
}

/* Input sample x_m: zero before the start unless a history of L-1 samples
 * (oldest first, so hist[L-2] is x_{-1}) is supplied. */
static void sample_at(const double *x, const double *hist, int32_t L, int64_t m,
                      double *re, double *im)
{
    if (m >= 0) {
        *re = x[2 * m];
        *im = x[2 * m + 1];
    } else if (hist && m >= -(int64_t)(L - 1)) {
        int64_t h = (int64_t)(L - 1) + m;
        *re = hist[2 * h];
        *im = hist[2 * h + 1];
    } else {
        *re = 0.0;
        *im = 0.0;
    }
}

/* |x|^(p-1) for odd p, by repeated multiplication of s = |x|^2 (low order to
 * high order, as section 3.2.1 describes). */
static double radial(int32_t p, double s)
{
    double r = 1.0;
    for (int32_t i = 0; i < (p - 1) / 2; ++i) r *= s;
    return r;
}

/* psi_p(x) = |x|^(p-1) x  (section 2.1, monomial form). */
static void psi(int32_t p, double re, double im, double *pr, double *pi)
{
    double s = re * re + im * im;
    double r = radial(p, s);
    *pr = r * re;
    *pi = r * im;
}

/* acc += w * v  (complex multiply-accumulate, written out). */
static void cmac(double *acc_r, double *acc_i, double wr, double wi, double vr, double vi)
{
    *acc_r += wr * vr - wi * vi;
    *acc_i += wr * vi + wi * vr;
}

/* One output z_n of Eq. (1): polynomial step, filtering step, accumulation + c. */
static void forward_one(const double *x, const double *hist, int64_t n,
                        const int32_t *mo, int32_t nm, const int32_t *co, int32_t nc,
                        int32_t L, const double *coeffs, double *zr, double *zi)
{
    double acc_r = 0.0, acc_i = 0.0;
    /* main branches: sum_p sum_k h_{p,k} psi_p(x_{n-k}) */
    for (int32_t b = 0; b < nm; ++b) {
        double fr = 0.0, fi = 0.0;                       /* f_p(x_n) */
        for (int32_t k = 0; k < L; ++k) {
            double xr, xi, pr, pi;
            sample_at(x, hist, L, n - k, &xr, &xi);
            psi(mo[b], xr, xi, &pr, &pi);
            const double *h = coeffs + 2 * ((int64_t)b * L + k);
            cmac(&fr, &fi, h[0], h[1], pr, pi);
        }
        acc_r += fr;
        acc_i += fi;
    }
    /* conjugate branches: sum_q sum_k hbar_{q,k} conj(psi_q(x_{n-k})) */
    for (int32_t b = 0; b < nc; ++b) {
        double fr = 0.0, fi = 0.0;                       /* f-bar_q(x_n) */
        for (int32_t k = 0; k < L; ++k) {
            double xr, xi, pr, pi;
            sample_at(x, hist, L, n - k, &xr, &xi);
            psi(co[b], xr, xi, &pr, &pi);
            const double *g = coeffs + 2 * ((int64_t)(nm + b) * L + k);
            cmac(&fr, &fi, g[0], g[1], pr, -pi);
        }
        acc_r += fr;
        acc_i += fi;
    }
    /* LO-leakage term c, the last coefficient */
    const double *c = coeffs + 2 * ((int64_t)(nm + nc) * L);
    *zr = acc_r + c[0];
    *zi = acc_i + c[1];
}

int oracle_forward(const double *x, int64_t n, const double *hist,
                   const int32_t *main_orders, int32_t n_main,
                   const int32_t *conj_orders, int32_t n_conj, int32_t L,
                   const double *coeffs, double *z)
{
    if (!check_args(n, main_orders, n_main, conj_orders, n_conj, L, coeffs)) return ORACLE_EINVAL;
    if (n > 0 && (!x || !z)) return ORACLE_EINVAL;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        forward_one(x, hist, i, main_orders, n_main, conj_orders, n_conj, L, coeffs,
                    &z[2 * i], &z[2 * i + 1]);
    return ORACLE_OK;
}

int oracle_forward_at(const double *x, int64_t n, const double *hist,
                      const int32_t *main_orders, int32_t n_main,
                      const int32_t *conj_orders, int32_t n_conj, int32_t L,
                      const double *coeffs, const int64_t *idx, int64_t count, double *z)
{
    if (!check_args(n, main_orders, n_main, conj_orders, n_conj, L, coeffs)) return ORACLE_EINVAL;
    if (count < 0 || (count > 0 && (!idx || !z || !x))) return ORACLE_EINVAL;
    for (int64_t j = 0; j < count; ++j)
        if (idx[j] < 0 || idx[j] >= n) return ORACLE_EINVAL;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < count; ++j)
        forward_one(x, hist, idx[j], main_orders, n_main, conj_orders, n_conj, L, coeffs,
                    &z[2 * j], &z[2 * j + 1]);
    return ORACLE_OK;
}

/*
 * Backward pass (not in the paper; derived from Eq. (1)).
 *
 * Convention: for a real loss E and complex w = a + jb the gradient is
 * dE/da + j dE/db.  G_n is that gradient with respect to the output z_n.
 *
 * Coefficients (Eq. (1) is linear in them):
 *   grad h_{p,k}    = sum_n G_n conj(psi_p(x_{n-k}))
 *   grad hbar_{q,k} = sum_n G_n psi_q(x_{n-k})
 *   grad c          = sum_n G_n
 * Input, with J = (p-1)/2, s = |x|^2 and the Wirtinger derivatives
 *   d psi_p / dx = (J+1) s^J,   d psi_p / dx* = J s^(J-1) x^2 :
 *   grad x_m = sum_{k} [ conj(G_{m+k}) dz_{m+k}/dx_m* + G_{m+k} conj(dz_{m+k}/dx_m) ]
 * with outputs beyond n-1 contributing nothing.  History samples are constants.
 */
static void dpsi(int32_t p, double xr, double xi, double *d_r, double *dc_r, double *dc_i)
{
    /* returns d psi/dx (real) and d psi/dx* (complex) */
    int32_t J = (p - 1) / 2;
    double s = xr * xr + xi * xi;
    *d_r = (double)(J + 1) * radial(p, s);
    if (J == 0) {
        *dc_r = 0.0;
        *dc_i = 0.0;
    } else {
        double r = (double)J * radial(p - 2, s);   /* J s^(J-1) */
        double x2r = xr * xr - xi * xi, x2i = 2.0 * xr * xi;
        *dc_r = r * x2r;
        *dc_i = r * x2i;
    }
}

static void backward_dx_one(const double *x, int64_t n, const int32_t *mo, int32_t nm,
                            const int32_t *co, int32_t nc, int32_t L, const double *coeffs,
                            const double *G, int64_t m, double *gr, double *gi)
{
    double xr = x[2 * m], xi = x[2 * m + 1];
    double sr = 0.0, si = 0.0;
    for (int32_t k = 0; k < L; ++k) {
        int64_t t = m + k;
        if (t >= n) break;
        /* dz_t/dx_m (A) and dz_t/dx_m* (B) */
        double Ar = 0.0, Ai = 0.0, Br = 0.0, Bi = 0.0;
        for (int32_t b = 0; b < nm; ++b) {
            double d, dcr, dci;
            dpsi(mo[b], xr, xi, &d, &dcr, &dci);
            const double *h = coeffs + 2 * ((int64_t)b * L + k);
            cmac(&Ar, &Ai, h[0], h[1], d, 0.0);
            cmac(&Br, &Bi, h[0], h[1], dcr, dci);
        }
        for (int32_t b = 0; b < nc; ++b) {
            double d, dcr, dci;
            dpsi(co[b], xr, xi, &d, &dcr, &dci);
            const double *g = coeffs + 2 * ((int64_t)(nm + b) * L + k);
            /* conj(psi): d/dx = conj(d psi/dx*),  d/dx* = conj(d psi/dx) = d */
            cmac(&Ar, &Ai, g[0], g[1], dcr, -dci);
            cmac(&Br, &Bi, g[0], g[1], d, 0.0);
        }
        double Gr = G[2 * t], Gi = G[2 * t + 1];
        cmac(&sr, &si, Gr, -Gi, Br, Bi);      /* conj(G) * B */
        cmac(&sr, &si, Gr, Gi, Ar, -Ai);      /* G * conj(A) */
    }
    *gr = sr;
    *gi = si;
}

int oracle_backward(const double *x, int64_t n, const double *hist,
                    const int32_t *main_orders, int32_t n_main,
                    const int32_t *conj_orders, int32_t n_conj, int32_t L,
                    const double *coeffs, const double *G, double *gx, double *gcoef)
{
    if (!check_args(n, main_orders, n_main, conj_orders, n_conj, L, coeffs)) return ORACLE_EINVAL;
    if (n > 0 && (!x || !G)) return ORACLE_EINVAL;
    const int64_t K = (int64_t)(n_main + n_conj) * L + 1;

    if (gx) {
#pragma omp parallel for schedule(static)
        for (int64_t m = 0; m < n; ++m)
            backward_dx_one(x, n, main_orders, n_main, conj_orders, n_conj, L, coeffs, G, m,
                            &gx[2 * m], &gx[2 * m + 1]);
    }
    if (gcoef) {
        /* one coefficient per task; each sum runs over n in increasing order */
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t kk = 0; kk < K; ++kk) {
            double ar = 0.0, ai = 0.0;
            if (kk == K - 1) {
                for (int64_t t = 0; t < n; ++t) {
                    ar += G[2 * t];
                    ai += G[2 * t + 1];
                }
            } else {
                int64_t branch = kk / L;
                int32_t k = (int32_t)(kk % L);
                int is_conj = branch >= n_main;
                int32_t p = is_conj ? conj_orders[branch - n_main] : main_orders[branch];
                for (int64_t t = 0; t < n; ++t) {
                    double xr, xi, pr, pi;
                    sample_at(x, hist, L, t - k, &xr, &xi);
                    psi(p, xr, xi, &pr, &pi);
                    if (is_conj)
                        cmac(&ar, &ai, G[2 * t], G[2 * t + 1], pr, pi);    /* G psi */
                    else
                        cmac(&ar, &ai, G[2 * t], G[2 * t + 1], pr, -pi);   /* G conj(psi) */
                }
            }
            gcoef[2 * kk] = ar;
            gcoef[2 * kk + 1] = ai;
        }
    }
    return ORACLE_OK;
}

/*
 * Normal equations of the least-squares estimate of section 2.2:
 *   A = Psi^H Psi  (K x K, Hermitian),  b = Psi^H t,
 * where row m of Psi is [psi_p(y_{m-k}) ..., conj(psi_q(y_{m-k})) ..., 1] for the
 * first M rows of the zero-filled element matrices of Eq. (2) (the L-1 tail rows
 * are dropped, matching an output of M samples), and t is the target sequence.
 * A is row-major, 2*K*K doubles; b is 2*K doubles.
 */
/* Row m of Psi (K complex entries, section 2.2 stacking) into row[]. */
static void ls_row(const double *y, int64_t m, const int32_t *mo, int32_t nm, const int32_t *co,
                   int32_t nc, int32_t L, double *row)
{
    int64_t col = 0;
    for (int32_t br = 0; br < nm + nc; ++br) {
        int is_conj = br >= nm;
        int32_t p = is_conj ? co[br - nm] : mo[br];
        for (int32_t k = 0; k < L; ++k, ++col) {
            double xr, xi, pr, pi;
            sample_at(y, NULL, L, m - k, &xr, &xi);
            psi(p, xr, xi, &pr, &pi);
            row[2 * col] = pr;
            row[2 * col + 1] = is_conj ? -pi : pi;
        }
    }
    row[2 * col] = 1.0;
    row[2 * col + 1] = 0.0;
}

int oracle_ls_normal(const double *y, int64_t M, const int32_t *main_orders, int32_t n_main,
                     const int32_t *conj_orders, int32_t n_conj, int32_t L,
                     const double *t, double *A, double *b)
{
    if (M < 0 || L < 1 || !check_orders(main_orders, n_main) || !check_orders(conj_orders, n_conj))
        return ORACLE_EINVAL;
    if (!A || !b || (M > 0 && (!y || !t))) return ORACLE_EINVAL;
    const int64_t K = (int64_t)(n_main + n_conj) * L + 1;
    memset(A, 0, sizeof(double) * 2 * (size_t)(K * K));
    memset(b, 0, sizeof(double) * 2 * (size_t)K);
    int failed = 0;
    /* Threads take bands of rows i of A (and entries of b); every entry is one
       sum over m in increasing order, so the result does not depend on the
       thread count. */
#pragma omp parallel
    {
        double *row = (double *)malloc(sizeof(double) * 2 * (size_t)K);
        if (!row) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t i0 = 0; i0 < K; i0 += 4) {
            if (!row) continue;
            const int64_t i1 = i0 + 4 < K ? i0 + 4 : K;
            for (int64_t m = 0; m < M; ++m) {
                ls_row(y, m, main_orders, n_main, conj_orders, n_conj, L, row);
                for (int64_t i = i0; i < i1; ++i) {
                    /* conj(row_i) * row_j and conj(row_i) * t_m */
                    double ir = row[2 * i], ii = -row[2 * i + 1];
                    for (int64_t j = 0; j < K; ++j)
                        cmac(&A[2 * (i * K + j)], &A[2 * (i * K + j) + 1], ir, ii, row[2 * j], row[2 * j + 1]);
                    cmac(&b[2 * i], &b[2 * i + 1], ir, ii, t[2 * m], t[2 * m + 1]);
                }
            }
        }
        free(row);
    }
    return failed ? ORACLE_EINVAL : ORACLE_OK;
}
