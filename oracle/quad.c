/*
 * CPU ORACLE -- test infrastructure only.  Nothing in the product library
 * links or calls this file; only tests, the smoke check and the benchmark's
 * CPU-baseline leg load it.
 *
 * Adaptive Gauss-Kronrod quadrature of the one-dimensional squared-
 * exponential kernel and its derivatives, integrated over cells.  This is the
 * plain definition of the 1-D building blocks of the GP-FVM Gram matrix
 * (Sec. 3.1 eq. linop-def-univariate and Sec. 3.2 eq. LkL): for intervals
 * I = [a,b], I' = [a2,b2]
 *
 *     F^{pq}(I,I') = int_I int_I' d^p/ds^p d^q/ds'^q k(s,s') ds' ds
 *     Q^{pq}(x,I') = int_I' d^p/dx^p d^q/ds'^q k(x,s') ds'
 *     P^{pq}(x,x') = d^p/dx^p d^q/dx'^q k(x,x')
 *
 * for the squared-exponential kernel k(s,s') = exp(-(s-s')^2 / (2 l^2))
 * (kq = -1) and for the half-integer Matern kernels (Sec. 3.1: nu = kq + 1/2,
 * k(r) = exp(-c |r| / l) p_kq(c |r| / l) with c = sqrt(2 kq + 1)).  No
 * antiderivative, no erf and no fundamental-theorem-of-calculus reduction is
 * used here: the derivative is evaluated pointwise -- for SE from the Hermite
 * representation
 *
 *     d^m/dr^m exp(-z^2) |_{z = r/(sqrt2 l)} = (-1/(sqrt2 l))^m H_m(z) e^{-z^2}
 *
 * (physicists' Hermite polynomials, three-term recurrence), for Matern by the
 * Leibniz rule on exp(-s) p(s) -- and the chain rule d/ds' = -d/dr for
 * r = s - s'.  The integrals are computed by recursive bisection with the
 * 7-point Gauss / 15-point Kronrod pair (QUADPACK's QK15 rule), nested for the
 * double integral; for Matern the panels are split where the integrand is not
 * smooth (r = 0, hence s' = s inside a cell and s at the ends of the inner
 * cell).
 */
#include <math.h>
#include <stddef.h>

/* Kronrod nodes (positive half), Kronrod weights, Gauss-7 weights. */
static const double XGK[8] = {
    0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
    0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
    0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
    0.207784955007898467600689403773245, 0.000000000000000000000000000000000};
static const double WGK[8] = {
    0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
    0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
    0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
    0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
/* Gauss weights for the Kronrod nodes of odd index 1,3,5 and the centre 7. */
static const double WG[4] = {
    0.129484966168869693270611432679082, 0.279705391489276667901467771423780,
    0.381830050505118944950369775488975, 0.417959183673469387755102040816327};

/* m-th derivative in r of exp(-r^2/(2 l^2)), m >= 0. */
double ora_kder(int m, double r, double ell)
{
    const double c = 1.0 / (sqrt(2.0) * ell);
    const double z = r * c;
    double h0 = 1.0, h1 = 2.0 * z, hm;
    if (m == 0) hm = h0;
    else if (m == 1) hm = h1;
    else {
        for (int n = 1; n < m; ++n) {
            double h2 = 2.0 * z * h1 - 2.0 * n * h0;
            h0 = h1; h1 = h2;
        }
        hm = h1;
    }
    double s = 1.0;
    for (int i = 0; i < m; ++i) s *= -c;
    return s * hm * exp(-z * z);
}

/* Coefficients of p_kq (Rasmussen & Williams eq. 4.16 written in s = c r / l):
 * p_kq(s) = kq!/(2kq)! sum_{i=0}^{kq} (kq+i)!/(i! (kq-i)!) (2s)^(kq-i). */
static void matern_poly(int kq, double* coef)
{
    double f[16];
    f[0] = 1.0;
    for (int i = 1; i < 16; ++i) f[i] = f[i - 1] * i;
    for (int k = 0; k <= kq; ++k) coef[k] = 0.0;
    for (int i = 0; i <= kq; ++i) {
        const int deg = kq - i;
        coef[deg] += f[kq] / f[2 * kq] * f[kq + i] / (f[i] * f[kq - i]) * pow(2.0, deg);
    }
}

/* m-th derivative in r of the Matern-(kq+1/2) kernel, m >= 0, by the Leibniz
 * rule on exp(-s) p(s), s = c |r| / l; even in r, so odd derivatives flip sign
 * for r < 0 and vanish at r = 0. */
double ora_kder_matern(int kq, int m, double r, double ell)
{
    double p[8], binom = 1.0, acc = 0.0;
    matern_poly(kq, p);
    const double c = sqrt(2.0 * kq + 1.0);
    const double s = c * fabs(r) / ell;
    for (int j = 0; j <= m; ++j) {
        /* j-th derivative of p at s */
        double dj = 0.0;
        for (int k = j; k <= kq; ++k) {
            double fall = 1.0;
            for (int t = 0; t < j; ++t) fall *= (double)(k - t);
            dj += p[k] * fall * pow(s, k - j);
        }
        const double sign = ((m - j) & 1) ? -1.0 : 1.0;
        acc += binom * sign * dj;
        binom = binom * (m - j) / (j + 1);
    }
    double v = acc * exp(-s) * pow(c / ell, m);
    if (m & 1) {
        if (r < 0) v = -v;
        else if (r == 0) v = 0.0;
    }
    return v;
}

/* kq < 0: squared exponential; kq >= 0: Matern nu = kq + 1/2. */
double ora_kder_k(int kq, int m, double r, double ell)
{
    return kq < 0 ? ora_kder(m, r, ell) : ora_kder_matern(kq, m, r, ell);
}

/* d^p/dx^p d^q/dx'^q k(x, x'); r = x - x', each d/dx' contributes -d/dr. */
double ora_point_point(int kq, int p, int q, double x, double x2, double ell)
{
    double v = ora_kder_k(kq, p + q, x - x2, ell);
    return (q & 1) ? -v : v;
}

typedef double (*integrand_t)(double s, const void* ctx);

static void qk15(integrand_t f, const void* ctx, double a, double b,
                 double* res_k, double* res_g, double* res_abs)
{
    const double c = 0.5 * (a + b), h = 0.5 * (b - a);
    double fc = f(c, ctx);
    double rk = fc * WGK[7], rg = fc * WG[3], ra = fabs(fc) * WGK[7];
    for (int j = 0; j < 7; ++j) {
        double dx = h * XGK[j];
        double f1 = f(c - dx, ctx), f2 = f(c + dx, ctx);
        rk += WGK[j] * (f1 + f2);
        ra += WGK[j] * (fabs(f1) + fabs(f2));
        if (j & 1) rg += WG[j >> 1] * (f1 + f2);
    }
    *res_k = rk * h; *res_g = rg * h; *res_abs = ra * fabs(h);
}

static double adapt(integrand_t f, const void* ctx, double a, double b,
                    double tol, int depth, long* budget)
{
    double k, g, ab;
    qk15(f, ctx, a, b, &k, &g, &ab);
    --*budget;
    /* accept on the requested tolerance, or once the Kronrod-Gauss gap is at
       the rounding level of this panel (further bisection cannot help), or
       when the depth or the panel budget of this integral is spent. */
    if (fabs(k - g) <= tol || fabs(k - g) <= 50.0 * 2.220446049250313e-16 * ab ||
        depth >= 30 || *budget <= 0)
        return k;
    const double m = 0.5 * (a + b);
    return adapt(f, ctx, a, m, 0.5 * tol, depth + 1, budget) +
           adapt(f, ctx, m, b, 0.5 * tol, depth + 1, budget);
}

/* Integral of f over [a,b], to absolute error ~ rel * int |f| (plus a floor);
   at most 4096 QK15 panels. */
static double integrate(integrand_t f, const void* ctx, double a, double b, double rel)
{
    if (a == b) return 0.0;
    double k, g, ab;
    qk15(f, ctx, a, b, &k, &g, &ab);
    double tol = rel * ab;
    if (tol < 1e-300) tol = 1e-300;
    long budget = 4096;
    return adapt(f, ctx, a, b, tol, 0, &budget);
}

typedef struct { int kq; int m; double x; double ell; double sign; } pc_ctx;

/* integrand s' -> d^p/dx^p d^q/ds'^q k(x, s') with m = p + q folded in. */
static double pc_f(double s2, const void* vc)
{
    const pc_ctx* c = (const pc_ctx*)vc;
    return c->sign * ora_kder_k(c->kq, c->m, c->x - s2, c->ell);
}

static const double REL_INNER = 1e-14;
static const double REL_OUTER = 1e-14;
static const double REL_OUTER_MATERN = 1e-12;

/* Integral over [a,b] split at the points of cuts[] that fall inside. */
static double integrate_split(integrand_t f, const void* ctx, double a, double b, double rel,
                              const double* cuts, int ncut)
{
    double pts[4];
    int n = 0;
    pts[n++] = a;
    for (int k = 0; k < ncut; ++k)
        if (cuts[k] > pts[n - 1] && cuts[k] < b) pts[n++] = cuts[k];
    double v = 0.0;
    for (int k = 0; k < n; ++k) v += integrate(f, ctx, pts[k], k + 1 < n ? pts[k + 1] : b, rel);
    return v;
}

double ora_point_cell(int kq, int p, int q, double x, double a2, double b2, double ell)
{
    pc_ctx c = {kq, p + q, x, ell, (q & 1) ? -1.0 : 1.0};
    return integrate_split(pc_f, &c, a2, b2, REL_INNER, &x, kq >= 0 ? 1 : 0);
}

typedef struct { int kq, p, q; double a2, b2, ell; } cc_ctx;

static double cc_f(double s, const void* vc)
{
    const cc_ctx* c = (const cc_ctx*)vc;
    return ora_point_cell(c->kq, c->p, c->q, s, c->a2, c->b2, c->ell);
}

double ora_cell_cell(int kq, int p, int q, double a, double b, double a2, double b2, double ell)
{
    cc_ctx c = {kq, p, q, a2, b2, ell};
    const double cuts[2] = {a2 < b2 ? a2 : b2, a2 < b2 ? b2 : a2};
    /* for Matern the inner integral is split at the moving kink, so its value
       carries rounding noise near 1e-14: the outer rule asks for less */
    return integrate_split(cc_f, &c, a, b, kq >= 0 ? REL_OUTER_MATERN : REL_OUTER, cuts, kq >= 0 ? 2 : 0);
}

/* Generic integral of d^m k(r) over [a,b] in r (used to pin the rule). */
typedef struct { int kq; int m; double ell; } r_ctx;
static double r_f(double r, const void* vc)
{
    const r_ctx* c = (const r_ctx*)vc;
    return ora_kder_k(c->kq, c->m, r, c->ell);
}
double ora_integrate_kder(int kq, int m, double a, double b, double ell)
{
    r_ctx c = {kq, m, ell};
    const double zero = 0.0;
    return integrate_split(r_f, &c, a, b, 1e-14, &zero, kq >= 0 ? 1 : 0);
}

/* Polynomial x^k over [a,b] with a single QK15 panel (Kronrod and Gauss). */
void ora_qk15_monomial(int k, double a, double b, double* kron, double* gauss)
{
    const double c = 0.5 * (a + b), h = 0.5 * (b - a);
    double rk = pow(c, k) * WGK[7], rg = pow(c, k) * WG[3];
    for (int j = 0; j < 7; ++j) {
        double f1 = pow(c - h * XGK[j], k), f2 = pow(c + h * XGK[j], k);
        rk += WGK[j] * (f1 + f2);
        if (j & 1) rg += WG[j >> 1] * (f1 + f2);
    }
    *kron = rk * h; *gauss = rg * h;
}

/* ---- matrix builders (row-major outputs) --------------------------------- */

/* out[i*n2 + j] = F^{pq}([e1[i],e1[i+1]], [e2[j],e2[j+1]]) */
void ora_cell_cell_matrix(int kq, int p, int q, int n1, const double* e1, int n2,
                          const double* e2, double ell, double* out)
{
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n2; ++j)
            out[(size_t)i * n2 + j] = ora_cell_cell(kq, p, q, e1[i], e1[i + 1], e2[j], e2[j + 1], ell);
}

/* out[i*n2 + j] = Q^{pq}(x[i], [e2[j],e2[j+1]]) */
void ora_point_cell_matrix(int kq, int p, int q, int n1, const double* x, int n2,
                           const double* e2, double ell, double* out)
{
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n2; ++j)
            out[(size_t)i * n2 + j] = ora_point_cell(kq, p, q, x[i], e2[j], e2[j + 1], ell);
}

/* out[i*n2 + j] = P^{pq}(x[i], x2[j]) */
void ora_point_point_matrix(int kq, int p, int q, int n1, const double* x, int n2,
                            const double* x2, double ell, double* out)
{
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n2; ++j)
            out[(size_t)i * n2 + j] = ora_point_point(kq, p, q, x[i], x2[j], ell);
}
