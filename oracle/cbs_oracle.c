/*
 * cbs_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the iterative Born solver for the
 * first-order acoustic system with heterogeneous sound speed, density and
 * absorption (arXiv 2507.16087).  It exists to check the GPU library against;
 * only the test-suite, the smoke check and the CPU-baseline timing may load it.
 * It shares no source with the GPU library (its own FFT, its own operator
 * assembly, its own shift selection).
 *
 * What it follows, by section of the paper:
 *  - complex sound speed, eq. (complex_sound_speed):  1/(rho c_cx^2) =
 *    (1 - 2 i alpha c / omega) / (rho c^2)                       -> field q
 *  - row-scaled first-order system, eq. (HH1stOrderSH), on the staggered grid
 *    of App. B.1: velocity component u_eta lives at x + dx/2 e_eta, the
 *    staggered density is the two-point average of rho, the absorbing rate is
 *    evaluated at the staggered points, and the off-diagonal operators are the
 *    spectral derivatives with the half-cell shift factor exp(+-i k dx/2).
 *  - split L + V with complex shifts a1, a2 and scaling C = diag(lam1, lam2),
 *    eqs. (LV) and (C); shifts as the centre of the minimum enclosing circle
 *    of each diagonal's values (Discussion) or the component-wise median
 *    (Algorithm 1 preprocessing).
 *  - (L+I)^{-1} per wavevector: the explicit staggered 3-D matrix of App. B.1
 *    (and its 2-D / 1-D restriction); the adjoint uses the per-k conjugate
 *    transpose of that matrix.
 *  - Algorithm 1: x = 0; repeat z = (L+I)^{-1}(B x + y),
 *    x <- x + nu B (z - x); stop when |x_{k+1} - x_k| / |x_k| <= tol; output
 *    C^{-1/2} x.
 *  - adjoint operator A^H (Sec. 2.3): the negated differential part plus the
 *    conjugated diagonal.
 *
 * Readings where the paper is silent or inconsistent: hat-sources s_p*q and
 * rhobar*s_u; absorbing layer
 * gamma = gmax * sum_eta r_eta^2 with r the periodic distance into the layer
 * over (L + 1/2); periodic wrap of the density average; scale floor
 * lam >= 1e-3 |a|; stopping test skipped at the first iteration.
 *
 * Collocated variant (App. B, first matrix): every field at the cell centres,
 * density and absorbing rate unshifted, derivative symbol i k with the
 * Nyquist bin of each odd derivative set to zero, (L+I)^{-1} the collocated
 * 3-D matrix (and its 2-D / 1-D restriction).
 *
 * Complex arrays are interleaved (re, im) doubles; fields are stored as
 * [F][cells] with F = ndim + 1 (u_0..u_{ndim-1}, p), C-ordered cells, last
 * axis contiguous.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ------------------------------------------------------------------------- */
/* FFT: recursive mixed-radix decimation in time, plain DFT for prime factors */
/* ------------------------------------------------------------------------- */

static int smallest_factor(int n)
{
    for (int p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

/* out[0..n) = DFT_n of in[0], in[stride], ...; tw[j] = exp(sign 2 pi i j / top)
 * and n divides top. */
static void fft_rec(const cplx *in, int n, int stride, cplx *out,
                    const cplx *tw, int top, cplx *tmp)
{
    if (n == 1) { out[0] = in[0]; return; }
    int p = smallest_factor(n), m = n / p;
    for (int r = 0; r < p; ++r)
        fft_rec(in + (size_t)r * stride, m, stride * p, out + (size_t)r * m, tw, top, tmp);
    int step = top / n;
    if (p == 2) {   /* X[k] = Y0 + w^k Y1, X[k + m] = Y0 - w^k Y1 */
        for (int k = 0; k < m; ++k) {
            cplx a = out[k], b = out[m + k] * tw[(size_t)k * step];
            out[k] = a + b;
            out[m + k] = a - b;
        }
        return;
    }
    /* X[k + m s] = sum_r w_n^{r k} Y_r[k] w_p^{r s} */
    for (int k = 0; k < m; ++k) {
        for (int r = 0; r < p; ++r)
            tmp[r] = out[(size_t)r * m + k] * tw[((size_t)r * k % n) * step];
        for (int s = 0; s < p; ++s) {
            cplx acc = 0;
            for (int r = 0; r < p; ++r)
                acc += tmp[r] * tw[((size_t)r * s * m % n) * step];
            out[(size_t)s * m + k] = acc;
        }
    }
}

/* Unnormalised DFT along every axis of a C-ordered complex array.
 * sign = -1 forward (exp(-i...)), +1 inverse. */
void orc_fft(int ndim, const int64_t *n, double *data_, int sign)
{
    cplx *data = (cplx *)data_;
    int64_t total = 1;
    for (int d = 0; d < ndim; ++d) total *= n[d];
    for (int ax = 0; ax < ndim; ++ax) {
        int len = (int)n[ax];
        if (len == 1) continue;
        int64_t stride = 1;
        for (int d = ax + 1; d < ndim; ++d) stride *= n[d];
        int64_t lines = total / len;
        cplx *tw = malloc(sizeof(cplx) * len);
        for (int j = 0; j < len; ++j) {
            double ang = sign * 2.0 * M_PI * (double)j / (double)len;
            tw[j] = cos(ang) + I * sin(ang);
        }
#pragma omp parallel
        {
            cplx *buf = malloc(sizeof(cplx) * len);
            cplx *res = malloc(sizeof(cplx) * len);
            cplx *tmp = malloc(sizeof(cplx) * len);
#pragma omp for schedule(static)
            for (int64_t l = 0; l < lines; ++l) {
                int64_t outer = l / stride, inner = l % stride;
                cplx *base = data + outer * stride * len + inner;
                for (int j = 0; j < len; ++j) buf[j] = base[(int64_t)j * stride];
                fft_rec(buf, len, 1, res, tw, len, tmp);
                for (int j = 0; j < len; ++j) base[(int64_t)j * stride] = res[j];
            }
            free(buf); free(res); free(tmp);
        }
        free(tw);
    }
}

/* ------------------------------------------------------------------------- */
/* minimum enclosing circle (Welzl, iterative, fixed pseudo-random order)     */
/* ------------------------------------------------------------------------- */

static void circle2(const double *a, const double *b, double *c, double *r)
{
    c[0] = 0.5 * (a[0] + b[0]); c[1] = 0.5 * (a[1] + b[1]);
    *r = 0.5 * hypot(a[0] - b[0], a[1] - b[1]);
}

static void circle3(const double *a, const double *b, const double *p, double *c, double *r)
{
    double bx = b[0] - a[0], by = b[1] - a[1], cx = p[0] - a[0], cy = p[1] - a[1];
    double d = 2.0 * (bx * cy - by * cx);
    if (fabs(d) < 1e-300) {            /* collinear: widest pair */
        double c1[2], c2[2], c3[2], r1, r2, r3;
        circle2(a, b, c1, &r1); circle2(a, p, c2, &r2); circle2(b, p, c3, &r3);
        if (r1 >= r2 && r1 >= r3) { c[0] = c1[0]; c[1] = c1[1]; *r = r1; }
        else if (r2 >= r3) { c[0] = c2[0]; c[1] = c2[1]; *r = r2; }
        else { c[0] = c3[0]; c[1] = c3[1]; *r = r3; }
        return;
    }
    double b2 = bx * bx + by * by, c2 = cx * cx + cy * cy;
    double ux = (cy * b2 - by * c2) / d, uy = (bx * c2 - cx * b2) / d;
    c[0] = a[0] + ux; c[1] = a[1] + uy;
    *r = hypot(ux, uy);
}

static int outside(const double *p, const double *c, double r)
{
    return hypot(p[0] - c[0], p[1] - c[1]) > r * (1.0 + 1e-12) + 1e-300;
}

/* pts: 2n doubles (x, y).  Result: centre (cx, cy), radius r. */
void orc_mec(const double *pts_in, int64_t n, double *out3)
{
    double *p = malloc(sizeof(double) * 2 * (size_t)n);
    memcpy(p, pts_in, sizeof(double) * 2 * (size_t)n);
    uint64_t s = 0x9E3779B97F4A7C15ull;
    for (int64_t i = n - 1; i > 0; --i) {      /* Fisher-Yates with an LCG */
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        int64_t j = (int64_t)((s >> 11) % (uint64_t)(i + 1));
        double tx = p[2 * i], ty = p[2 * i + 1];
        p[2 * i] = p[2 * j]; p[2 * i + 1] = p[2 * j + 1];
        p[2 * j] = tx; p[2 * j + 1] = ty;
    }
    double c[2] = {p[0], p[1]}, r = 0.0;
    for (int64_t i = 1; i < n; ++i) {
        if (!outside(p + 2 * i, c, r)) continue;
        c[0] = p[2 * i]; c[1] = p[2 * i + 1]; r = 0.0;
        for (int64_t j = 0; j < i; ++j) {
            if (!outside(p + 2 * j, c, r)) continue;
            circle2(p + 2 * i, p + 2 * j, c, &r);
            for (int64_t k = 0; k < j; ++k)
                if (outside(p + 2 * k, c, r)) circle3(p + 2 * i, p + 2 * j, p + 2 * k, c, &r);
        }
    }
    out3[0] = c[0]; out3[1] = c[1]; out3[2] = r;
    free(p);
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

static double median_of(double *v, int64_t n)
{
    qsort(v, (size_t)n, sizeof(double), cmp_double);
    return (n % 2) ? v[n / 2] : 0.5 * (v[n / 2 - 1] + v[n / 2]);
}

/* ------------------------------------------------------------------------- */
/* medium                                                                     */
/* ------------------------------------------------------------------------- */

typedef struct {
    int ndim;
    int64_t n[3];
    int64_t ncell;
    double dx, omega, gmax, beta, nu;
    int pml, shift_rule;
    int colloc;       /* 1: collocated grid variant                           */
    double *rho, *c, *alpha;
    cplx *q;          /* 1/(rho c_cx^2) per cell                               */
    double *rhobar;   /* [ndim][ncell] staggered density                       */
    double *gam;      /* absorbing rate at cell centres                        */
    double *gams;     /* [ndim][ncell] absorbing rate at staggered points      */
    cplx *Du;         /* [ndim][ncell] rhobar (i omega + gamma_eta)            */
    cplx *Dp;         /* (i omega + gamma) q                                   */
    cplx a1, a2;
    double lam1, lam2;
    double *kv[3];    /* wavenumbers per axis, FFT order                       */
    cplx *sh[3];      /* half-cell shift factors exp(i k dx/2) per axis        */
    double *kd[3];    /* collocated derivative wavenumbers (Nyquist bin 0)     */
} orc_medium;

/* periodic distance of position t from the interior [L, n-1-L], over L+1/2 */
static double layer_r(double t, int n, int L)
{
    if (L <= 0) return 0.0;
    double lo = L, hi = n - 1 - L;
    double d;
    if (t >= lo && t <= hi) return 0.0;
    if (t > hi) d = fmin(t - hi, lo + n - t);
    else d = fmin(lo - t, t + n - hi);
    return d / (L + 0.5);
}

static void unravel(int64_t idx, int ndim, const int64_t *n, int64_t *ix)
{
    for (int d = ndim - 1; d >= 0; --d) { ix[d] = idx % n[d]; idx /= n[d]; }
}

static int64_t neighbour(int64_t idx, int ndim, const int64_t *n, int axis, int delta)
{
    int64_t ix[3];
    unravel(idx, ndim, n, ix);
    ix[axis] = (ix[axis] + delta + n[axis]) % n[axis];
    int64_t out = 0;
    for (int d = 0; d < ndim; ++d) out = out * n[d] + ix[d];
    return out;
}

void orc_destroy(void *h)
{
    orc_medium *m = h;
    if (!m) return;
    free(m->rho); free(m->c); free(m->alpha); free(m->q); free(m->rhobar);
    free(m->gam); free(m->gams); free(m->Du); free(m->Dp);
    for (int d = 0; d < 3; ++d) { free(m->kv[d]); free(m->sh[d]); free(m->kd[d]); }
    free(m);
}

/* Returns 0 on success, -1 on invalid input.  colloc selects the collocated
 * variant. */
int orc_create2(int ndim, const int64_t *n, double dx, double omega, int pml,
                double gmax, double beta, double nu, int shift_rule, int colloc,
                const double *c, const double *rho, const double *alpha, void **out)
{
    *out = NULL;
    if (ndim < 1 || ndim > 3 || !(dx > 0) || !(omega > 0)) return -1;
    orc_medium *m = calloc(1, sizeof(orc_medium));
    m->ndim = ndim;
    m->ncell = 1;
    for (int d = 0; d < 3; ++d) m->n[d] = 1;
    for (int d = 0; d < ndim; ++d) {
        if (n[d] < 1) { free(m); return -1; }
        m->n[d] = n[d];
        m->ncell *= n[d];
        if (pml > 0 && 2 * pml >= n[d]) { free(m); return -1; }
    }
    m->dx = dx; m->omega = omega; m->pml = pml;
    m->gmax = gmax > 0 ? gmax : omega;
    m->beta = beta; m->nu = nu; m->shift_rule = shift_rule; m->colloc = colloc;
    int64_t N = m->ncell;
    for (int64_t i = 0; i < N; ++i)
        if (!(c[i] > 0) || !(rho[i] > 0) || !(alpha[i] >= 0) || !isfinite(c[i]) ||
            !isfinite(rho[i]) || !isfinite(alpha[i])) { free(m); return -1; }
    m->rho = malloc(sizeof(double) * N); memcpy(m->rho, rho, sizeof(double) * N);
    m->c = malloc(sizeof(double) * N); memcpy(m->c, c, sizeof(double) * N);
    m->alpha = malloc(sizeof(double) * N); memcpy(m->alpha, alpha, sizeof(double) * N);
    m->q = malloc(sizeof(cplx) * N);
    m->rhobar = malloc(sizeof(double) * ndim * N);
    m->gam = malloc(sizeof(double) * N);
    m->gams = malloc(sizeof(double) * ndim * N);
    m->Du = malloc(sizeof(cplx) * ndim * N);
    m->Dp = malloc(sizeof(cplx) * N);

    /* complex sound speed: 1/(rho c_cx^2) = (1 - 2 i alpha c / omega)/(rho c^2) */
    for (int64_t i = 0; i < N; ++i)
        m->q[i] = (1.0 - 2.0 * I * alpha[i] * c[i] / omega) / (rho[i] * c[i] * c[i]);

    /* absorbing rate at centres and at the staggered points */
    for (int64_t i = 0; i < N; ++i) {
        int64_t ix[3];
        unravel(i, ndim, m->n, ix);
        double g = 0.0;
        for (int d = 0; d < ndim; ++d) {
            double r = layer_r((double)ix[d], (int)m->n[d], pml);
            g += r * r;
        }
        m->gam[i] = m->gmax * g;
        for (int e = 0; e < ndim; ++e) {
            double gs = 0.0;
            for (int d = 0; d < ndim; ++d) {
                double t = (double)ix[d] + ((d == e && !colloc) ? 0.5 : 0.0);
                double r = layer_r(t, (int)m->n[d], pml);
                gs += r * r;
            }
            m->gams[(size_t)e * N + i] = m->gmax * gs;
        }
    }
    /* staggered density: average of rho at x and x + dx e_eta (periodic) */
    for (int e = 0; e < ndim; ++e)
        for (int64_t i = 0; i < N; ++i)
            m->rhobar[(size_t)e * N + i] = colloc ? rho[i]
                                                  : 0.5 * (rho[i] + rho[neighbour(i, ndim, m->n, e, +1)]);

    /* diagonal blocks of the row-scaled staggered system */
    for (int e = 0; e < ndim; ++e)
        for (int64_t i = 0; i < N; ++i)
            m->Du[(size_t)e * N + i] = m->rhobar[(size_t)e * N + i] *
                                       (I * omega + m->gams[(size_t)e * N + i]);
    for (int64_t i = 0; i < N; ++i)
        m->Dp[i] = (I * omega + m->gam[i]) * m->q[i];

    /* complex shifts */
    int64_t nu_pts = (int64_t)ndim * N;
    if (shift_rule == 1) {
        double *v = malloc(sizeof(double) * nu_pts);
        for (int64_t i = 0; i < nu_pts; ++i) v[i] = creal(m->Du[i]);
        double re = median_of(v, nu_pts);
        for (int64_t i = 0; i < nu_pts; ++i) v[i] = cimag(m->Du[i]);
        m->a1 = re + I * median_of(v, nu_pts);
        for (int64_t i = 0; i < N; ++i) v[i] = creal(m->Dp[i]);
        re = median_of(v, N);
        for (int64_t i = 0; i < N; ++i) v[i] = cimag(m->Dp[i]);
        m->a2 = re + I * median_of(v, N);
        free(v);
    } else {
        double res[3];
        orc_mec((const double *)m->Du, nu_pts, res);
        m->a1 = res[0] + I * res[1];
        orc_mec((const double *)m->Dp, N, res);
        m->a2 = res[0] + I * res[1];
    }
    /* scaling: lam = max |D - a| / beta, floored at 1e-3 |a| */
    double r1 = 0.0, r2 = 0.0;
    for (int64_t i = 0; i < nu_pts; ++i) r1 = fmax(r1, cabs(m->Du[i] - m->a1));
    for (int64_t i = 0; i < N; ++i) r2 = fmax(r2, cabs(m->Dp[i] - m->a2));
    m->lam1 = fmax(r1, 1e-3 * cabs(m->a1)) / beta;
    m->lam2 = fmax(r2, 1e-3 * cabs(m->a2)) / beta;

    for (int d = 0; d < 3; ++d) {
        int len = (int)m->n[d];
        m->kv[d] = malloc(sizeof(double) * len);
        for (int j = 0; j < len; ++j) {
            int f = (j < (len + 1) / 2) ? j : j - len;   /* numpy fftfreq order */
            m->kv[d][j] = (d < ndim) ? 2.0 * M_PI * f / (len * dx) : 0.0;
        }
        m->sh[d] = malloc(sizeof(cplx) * len);
        for (int j = 0; j < len; ++j) m->sh[d][j] = cexp(I * m->kv[d][j] * dx / 2.0);
        m->kd[d] = malloc(sizeof(double) * len);
        for (int j = 0; j < len; ++j)
            m->kd[d][j] = (len % 2 == 0 && j == len / 2) ? 0.0 : m->kv[d][j];
    }
    *out = m;
    return 0;
}

int orc_create(int ndim, const int64_t *n, double dx, double omega, int pml,
               double gmax, double beta, double nu, int shift_rule,
               const double *c, const double *rho, const double *alpha, void **out)
{
    return orc_create2(ndim, n, dx, omega, pml, gmax, beta, nu, shift_rule, 0, c, rho, alpha, out);
}

/* a1 (re, im), a2 (re, im), lam1, lam2, beta, nu */
void orc_get_scalars(void *h, double *o)
{
    orc_medium *m = h;
    o[0] = creal(m->a1); o[1] = cimag(m->a1); o[2] = creal(m->a2); o[3] = cimag(m->a2);
    o[4] = m->lam1; o[5] = m->lam2; o[6] = m->beta; o[7] = m->nu;
}

void orc_set_scalars(void *h, const double *s)
{
    orc_medium *m = h;
    m->a1 = s[0] + I * s[1]; m->a2 = s[2] + I * s[3]; m->lam1 = s[4]; m->lam2 = s[5];
}

void orc_set_nu(void *h, double nu) { ((orc_medium *)h)->nu = nu; }

/* q (complex), rhobar [ndim][N], gamma [N], gamma_staggered [ndim][N] */
void orc_get_fields(void *h, double *q, double *rhobar, double *gam, double *gams)
{
    orc_medium *m = h;
    int64_t N = m->ncell;
    if (q) memcpy(q, m->q, sizeof(cplx) * N);
    if (rhobar) memcpy(rhobar, m->rhobar, sizeof(double) * m->ndim * N);
    if (gam) memcpy(gam, m->gam, sizeof(double) * N);
    if (gams) memcpy(gams, m->gams, sizeof(double) * m->ndim * N);
}

/* ------------------------------------------------------------------------- */
/* operators                                                                  */
/* ------------------------------------------------------------------------- */

static void kvec(const orc_medium *m, int64_t idx, double *k, cplx *S)
{
    int64_t ix[3];
    unravel(idx, m->ndim, m->n, ix);
    for (int d = 0; d < m->ndim; ++d) { k[d] = m->kv[d][ix[d]]; S[d] = m->sh[d][ix[d]]; }
}

/* Physical row-scaled staggered operator A (or A^H):
 *   (A xi)_u_eta = D_u_eta u_eta + F^-1[ i k_eta S_eta   F p ]
 *   (A xi)_p     = D_p p         + sum_eta F^-1[ i k_eta S^eta F u_eta ]
 * with S_eta = exp(i k_eta dx/2) and S^eta its conjugate.  The adjoint
 * conjugates the diagonal and negates the differential part. */
int orc_apply_A(void *h, int adjoint, const double *xi_, double *out_)
{
    orc_medium *m = h;
    int D = m->ndim;
    int64_t N = m->ncell;
    const cplx *xi = (const cplx *)xi_;
    cplx *out = (cplx *)out_;
    cplx *sp = malloc(sizeof(cplx) * (D + 1) * N);
    memcpy(sp, xi, sizeof(cplx) * (D + 1) * N);
    for (int f = 0; f <= D; ++f) orc_fft(D, m->n, (double *)(sp + (size_t)f * N), -1);
    cplx *dr = calloc((size_t)(D + 1) * N, sizeof(cplx));
    double sgn = adjoint ? -1.0 : 1.0;
    for (int64_t i = 0; i < N; ++i) {
        double k[3];
        cplx S[3];
        kvec(m, i, k, S);
        cplx pp = sp[(size_t)D * N + i], acc = 0;
        if (m->colloc) {          /* i k, Nyquist bin of the odd derivative zeroed */
            int64_t ix[3];
            unravel(i, D, m->n, ix);
            for (int e = 0; e < D; ++e) {
                double kd = m->kd[e][ix[e]];
                dr[(size_t)e * N + i] = sgn * I * kd * pp;
                acc += sgn * I * kd * sp[(size_t)e * N + i];
            }
        } else {
            for (int e = 0; e < D; ++e) {
                dr[(size_t)e * N + i] = sgn * I * k[e] * S[e] * pp;
                acc += sgn * I * k[e] * conj(S[e]) * sp[(size_t)e * N + i];
            }
        }
        dr[(size_t)D * N + i] = acc;
    }
    for (int f = 0; f <= D; ++f) orc_fft(D, m->n, (double *)(dr + (size_t)f * N), +1);
    for (int e = 0; e < D; ++e)
        for (int64_t i = 0; i < N; ++i) {
            cplx d = adjoint ? conj(m->Du[(size_t)e * N + i]) : m->Du[(size_t)e * N + i];
            out[(size_t)e * N + i] = d * xi[(size_t)e * N + i] + dr[(size_t)e * N + i] / (double)N;
        }
    for (int64_t i = 0; i < N; ++i) {
        cplx d = adjoint ? conj(m->Dp[i]) : m->Dp[i];
        out[(size_t)D * N + i] = d * xi[(size_t)D * N + i] + dr[(size_t)D * N + i] / (double)N;
    }
    free(sp); free(dr);
    return 0;
}

/* Explicit (L+I)^{-1} of App. B.1 at one wavevector, (D+1)x(D+1), row-major.
 * Notation: alpha1 = a1 + lam1, mu = |k|^2 + (a1 + lam1)(a2 + lam2),
 * S_eta = exp(i k_eta dx/2), S^eta = conj(S_eta), S_eta^mu = S_eta S^mu. */
static void propagator(const orc_medium *m, const double *k, const cplx *S, cplx *M)
{
    int D = m->ndim, F = D + 1;
    cplx al1 = m->a1 + m->lam1, al2 = m->a2 + m->lam2;
    double kk = 0;
    for (int e = 0; e < D; ++e) kk += k[e] * k[e];
    cplx mu = kk + al1 * al2;
    double s = sqrt(m->lam1 * m->lam2);
    for (int e = 0; e < D; ++e) {
        for (int f = 0; f < D; ++f) {
            cplx Sef = S[e] * conj(S[f]);
            cplx v = (e == f) ? (mu - k[e] * k[e]) : -k[e] * k[f] * Sef;
            M[e * F + f] = m->lam1 * v / (al1 * mu);
        }
        M[e * F + D] = -I * k[e] * s * S[e] / mu;
        M[D * F + e] = -I * k[e] * s * conj(S[e]) / mu;
    }
    M[D * F + D] = m->lam2 * al1 / mu;
}

/* Collocated (L+I)^{-1} of App. B (first matrix) with k the collocated
 * derivative wavenumbers:
 *   M = (1/mu) [[ lam1/alpha1 (mu I - k k^T), -i s k ], [ -i s k^T, lam2 alpha1 ]]. */
static void propagator_colloc(const orc_medium *m, const double *k, cplx *M)
{
    int D = m->ndim, F = D + 1;
    cplx al1 = m->a1 + m->lam1, al2 = m->a2 + m->lam2;
    double kk = 0;
    for (int e = 0; e < D; ++e) kk += k[e] * k[e];
    cplx mu = kk + al1 * al2;
    double s = sqrt(m->lam1 * m->lam2);
    for (int e = 0; e < D; ++e) {
        for (int f = 0; f < D; ++f)
            M[e * F + f] = m->lam1 * ((e == f ? mu : 0.0) - k[e] * k[f]) / (al1 * mu);
        M[e * F + D] = -I * s * k[e] / mu;
        M[D * F + e] = -I * s * k[e] / mu;
    }
    M[D * F + D] = m->lam2 * al1 / mu;
}

static void propagator_any(const orc_medium *m, int64_t idx, cplx *M)
{
    double k[3];
    cplx S[3];
    kvec(m, idx, k, S);
    if (m->colloc) {
        int64_t ix[3];
        unravel(idx, m->ndim, m->n, ix);
        double kd[3];
        for (int e = 0; e < m->ndim; ++e) kd[e] = m->kd[e][ix[e]];
        propagator_colloc(m, kd, M);
    } else {
        propagator(m, k, S, M);
    }
}

/* Write the propagator at flat k index idx (for tests); adjoint gives M^H. */
void orc_propagator_at(void *h, int64_t idx, int adjoint, double *out_)
{
    orc_medium *m = h;
    int F = m->ndim + 1;
    cplx M[16], *out = (cplx *)out_;
    propagator_any(m, idx, M);
    for (int r = 0; r < F; ++r)
        for (int c = 0; c < F; ++c)
            out[r * F + c] = adjoint ? conj(M[c * F + r]) : M[r * F + c];
}

/* B = I - V, V = C^-1/2 (D - a) C^-1/2 (diagonal), conjugated for the adjoint */
static cplx Bval(const orc_medium *m, int f, int64_t i, int adjoint)
{
    int D = m->ndim;
    int64_t N = m->ncell;
    cplx b = (f < D) ? 1.0 - (m->Du[(size_t)f * N + i] - m->a1) / m->lam1
                     : 1.0 - (m->Dp[i] - m->a2) / m->lam2;
    return adjoint ? conj(b) : b;
}

/* Scaled split operator A_s = L + V = C^-1/2 A C^-1/2 applied to x. */
static void apply_As(orc_medium *m, int adjoint, const cplx *x, cplx *out)
{
    int D = m->ndim;
    int64_t N = m->ncell;
    cplx *xi = malloc(sizeof(cplx) * (D + 1) * N);
    for (int f = 0; f <= D; ++f) {
        double sc = 1.0 / sqrt(f < D ? m->lam1 : m->lam2);
        for (int64_t i = 0; i < N; ++i) xi[(size_t)f * N + i] = sc * x[(size_t)f * N + i];
    }
    orc_apply_A(m, adjoint, (const double *)xi, (double *)out);
    for (int f = 0; f <= D; ++f) {
        double sc = 1.0 / sqrt(f < D ? m->lam1 : m->lam2);
        for (int64_t i = 0; i < N; ++i) out[(size_t)f * N + i] *= sc;
    }
    free(xi);
}

/* Hat-source of the row-scaled system: s_u,eta * rhobar_eta and s_p * q. */
void orc_source_hat(void *h, const double *s_, double *shat_)
{
    orc_medium *m = h;
    int D = m->ndim;
    int64_t N = m->ncell;
    const cplx *s = (const cplx *)s_;
    cplx *shat = (cplx *)shat_;
    for (int e = 0; e < D; ++e)
        for (int64_t i = 0; i < N; ++i)
            shat[(size_t)e * N + i] = m->rhobar[(size_t)e * N + i] * s[(size_t)e * N + i];
    for (int64_t i = 0; i < N; ++i)
        shat[(size_t)D * N + i] = m->q[i] * s[(size_t)D * N + i];
}

/* Algorithm 1 on A xi = shat (adjoint: A^H xi = shat).
 *   y = C^-1/2 shat; x = 0;
 *   repeat: w = B x + y; z = F^-1 [ M(k) F w ]; x <- x + nu B (z - x)
 *   until |x_new - x| / |x| <= tol (tested from the second iteration on)
 *   xi = C^-1/2 x.
 * history (nullable, max_iter doubles) receives the relative update per
 * iteration (0 at the first).  Returns 0 converged, 1 iteration cap. */
int orc_solve(void *h, int adjoint, const double *shat_, double tol, int64_t max_iter,
              double *xi_out_, int64_t *iters, double *rel_update, double *history,
              const double *x0_)
{
    orc_medium *m = h;
    int D = m->ndim, F = D + 1;
    int64_t N = m->ncell;
    const cplx *shat = (const cplx *)shat_;
    cplx *y = malloc(sizeof(cplx) * F * N);
    cplx *x = calloc((size_t)F * N, sizeof(cplx));
    cplx *w = malloc(sizeof(cplx) * F * N);
    for (int f = 0; f < F; ++f) {
        double sc = 1.0 / sqrt(f < D ? m->lam1 : m->lam2);
        for (int64_t i = 0; i < N; ++i) y[(size_t)f * N + i] = sc * shat[(size_t)f * N + i];
    }
    if (x0_) {     /* resume from a previous scaled state (checkpoint) */
        const cplx *x0 = (const cplx *)x0_;
        for (int64_t i = 0; i < (int64_t)F * N; ++i) x[i] = x0[i];
    }
    int status = 1;
    int64_t it = 0;
    double rel = INFINITY;
    for (it = 0; it < max_iter; ++it) {
        for (int f = 0; f < F; ++f)
            for (int64_t i = 0; i < N; ++i)
                w[(size_t)f * N + i] = Bval(m, f, i, adjoint) * x[(size_t)f * N + i] +
                                       y[(size_t)f * N + i];
        for (int f = 0; f < F; ++f) orc_fft(D, m->n, (double *)(w + (size_t)f * N), -1);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            cplx M[16], v[4], r[4];
            propagator_any(m, i, M);
            for (int f = 0; f < F; ++f) v[f] = w[(size_t)f * N + i];
            for (int a = 0; a < F; ++a) {
                cplx acc = 0;
                for (int b = 0; b < F; ++b)
                    acc += (adjoint ? conj(M[b * F + a]) : M[a * F + b]) * v[b];
                r[a] = acc;
            }
            for (int f = 0; f < F; ++f) w[(size_t)f * N + i] = r[f];
        }
        for (int f = 0; f < F; ++f) orc_fft(D, m->n, (double *)(w + (size_t)f * N), +1);
        double dn = 0, on = 0;
        for (int f = 0; f < F; ++f)
            for (int64_t i = 0; i < N; ++i) {
                size_t j = (size_t)f * N + i;
                cplx z = w[j] / (double)N;
                cplx dxv = m->nu * Bval(m, f, i, adjoint) * (z - x[j]);
                on += creal(x[j]) * creal(x[j]) + cimag(x[j]) * cimag(x[j]);
                dn += creal(dxv) * creal(dxv) + cimag(dxv) * cimag(dxv);
                x[j] += dxv;
            }
        rel = (on > 0) ? sqrt(dn / on) : INFINITY;
        if (history) history[it] = (on > 0) ? rel : 0.0;
        if (on > 0 && rel <= tol) { ++it; status = 0; break; }
    }
    if (iters) *iters = it;
    if (rel_update) *rel_update = rel;
    cplx *xi_out = (cplx *)xi_out_;
    for (int f = 0; f < F; ++f) {
        double sc = 1.0 / sqrt(f < D ? m->lam1 : m->lam2);
        for (int64_t i = 0; i < N; ++i) xi_out[(size_t)f * N + i] = sc * x[(size_t)f * N + i];
    }
    free(y); free(x); free(w);
    return status;
}

/* Scaled residual |y - A_s x| / |y| of a physical solution xi for rhs shat. */
double orc_rel_residual(void *h, int adjoint, const double *shat_, const double *xi_)
{
    orc_medium *m = h;
    int D = m->ndim, F = D + 1;
    int64_t N = m->ncell;
    const cplx *shat = (const cplx *)shat_, *xi = (const cplx *)xi_;
    cplx *x = malloc(sizeof(cplx) * F * N), *ax = malloc(sizeof(cplx) * F * N);
    for (int f = 0; f < F; ++f) {
        double sc = sqrt(f < D ? m->lam1 : m->lam2);
        for (int64_t i = 0; i < N; ++i) x[(size_t)f * N + i] = sc * xi[(size_t)f * N + i];
    }
    apply_As(m, adjoint, x, ax);
    double rn = 0, yn = 0;
    for (int f = 0; f < F; ++f) {
        double sc = 1.0 / sqrt(f < D ? m->lam1 : m->lam2);
        for (int64_t i = 0; i < N; ++i) {
            cplx yv = sc * shat[(size_t)f * N + i];
            cplx r = yv - ax[(size_t)f * N + i];
            rn += creal(r) * creal(r) + cimag(r) * cimag(r);
            yn += creal(yv) * creal(yv) + cimag(yv) * cimag(yv);
        }
    }
    free(x); free(ax);
    return sqrt(rn / yn);
}

/* Misfit gradient for a real parameter field from the forward solution xi of
 * A xi = shat(s) and the adjoint solution lam of A^H lam = g:
 *   dJ/dm(x) = Re sum_rows conj(lam_row) [ d shat_row/dm(x) - dD_row/dm(x) xi_row ]
 * with D_p = (i w + gamma) q, q = (1 - 2 i alpha c/w)/(rho c^2),
 * D_u_eta = rhobar_eta (i w + gamma_eta), rhobar_eta = (rho(x) + rho(x+e_eta))/2,
 * shat_p = q s_p, shat_u_eta = rhobar_eta s_u_eta.
 * s: physical source [F][N] complex (velocity rows may be zero). */
void orc_gradient(void *h, const double *s_, const double *xi_, const double *lam_,
                  double *gc, double *grho, double *galpha)
{
    orc_medium *m = h;
    int D = m->ndim;
    int64_t N = m->ncell;
    const cplx *s = (const cplx *)s_, *xi = (const cplx *)xi_, *lam = (const cplx *)lam_;
    double w = m->omega;
    for (int64_t i = 0; i < N; ++i) {
        double c = m->c[i], rho = m->rho[i], al = m->alpha[i];
        cplx q = m->q[i];
        cplx dq_dc = (-2.0 / (c * c * c) + 2.0 * I * al / (w * c * c)) / rho;
        cplx dq_drho = -q / rho;
        cplx dq_dal = -2.0 * I / (w * rho * c);
        size_t ip = (size_t)D * N + i;
        /* pressure row: shat_p - D_p p = q (s_p - (i w + gamma) p) */
        cplx core = conj(lam[ip]) * (s[ip] - (I * w + m->gam[i]) * xi[ip]);
        gc[i] = creal(core * dq_dc);
        galpha[i] = creal(core * dq_dal);
        double gr = creal(core * dq_drho);
        /* velocity rows: rhobar_eta at x and at x - e_eta depend on rho(x)
         * (collocated: the velocity rows at x only, weight 1) */
        for (int e = 0; e < D; ++e) {
            if (m->colloc) {
                size_t a = (size_t)e * N + i;
                gr += creal(conj(lam[a]) * (s[a] - (I * w + m->gams[a]) * xi[a]));
                continue;
            }
            int64_t j = neighbour(i, D, m->n, e, -1);
            size_t a = (size_t)e * N + i, b = (size_t)e * N + j;
            cplx ta = conj(lam[a]) * (s[a] - (I * w + m->gams[a]) * xi[a]);
            cplx tb = conj(lam[b]) * (s[b] - (I * w + m->gams[b]) * xi[b]);
            gr += 0.5 * creal(ta) + 0.5 * creal(tb);
        }
        grho[i] = gr;
    }
}
