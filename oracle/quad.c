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
 * with k(s,s') = exp(-(s-s')^2 / (2 l^2)).  No antiderivative, no erf and no
 * fundamental-theorem-of-calculus reduction is used here: the derivative is
 * evaluated pointwise from the Hermite representation
 *
 *     d^m/dr^m exp(-z^2) |_{z = r/(sqrt2 l)} = (-1/(sqrt2 l))^m H_m(z) e^{-z^2}
 *
 * (physicists' Hermite polynomials, three-term recurrence) and the chain rule
 * d/ds' = -d/dr for r = s - s'.  The integrals are computed by recursive
 * bisection with the 7-point Gauss / 15-point Kronrod pair (QUADPACK's QK15
 * rule), nested for the double integral.
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

/* d^p/dx^p d^q/dx'^q k(x, x'); r = x - x', each d/dx' contributes -d/dr. */
double ora_point_point(int p, int q, double x, double x2, double ell)
{
    double v = ora_kder(p + q, x - x2, ell);
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
                    double tol, int depth)
{
    double k, g, ab;
    qk15(f, ctx, a, b, &k, &g, &ab);
    /* accept on the requested tolerance, or once the Kronrod-Gauss gap is at
       the rounding level of this panel (further bisection cannot help). */
    if (fabs(k - g) <= tol || fabs(k - g) <= 50.0 * 2.220446049250313e-16 * ab ||
        depth >= 30)
        return k;
    const double m = 0.5 * (a + b);
    return adapt(f, ctx, a, m, 0.5 * tol, depth + 1) +
           adapt(f, ctx, m, b, 0.5 * tol, depth + 1);
}

/* Integral of f over [a,b], to absolute error ~ rel * int |f| (plus a floor). */
static double integrate(integrand_t f, const void* ctx, double a, double b, double rel)
{
    if (a == b) return 0.0;
    double k, g, ab;
    qk15(f, ctx, a, b, &k, &g, &ab);
    double tol = rel * ab;
    if (tol < 1e-300) tol = 1e-300;
    return adapt(f, ctx, a, b, tol, 0);
}

typedef struct { int m; double x; double ell; double sign; } pc_ctx;

/* integrand s' -> d^p/dx^p d^q/ds'^q k(x, s') with m = p + q folded in. */
static double pc_f(double s2, const void* vc)
{
    const pc_ctx* c = (const pc_ctx*)vc;
    return c->sign * ora_kder(c->m, c->x - s2, c->ell);
}

static const double REL_INNER = 1e-14;
static const double REL_OUTER = 1e-14;

double ora_point_cell(int p, int q, double x, double a2, double b2, double ell)
{
    pc_ctx c = {p + q, x, ell, (q & 1) ? -1.0 : 1.0};
    return integrate(pc_f, &c, a2, b2, REL_INNER);
}

typedef struct { int p, q; double a2, b2, ell; } cc_ctx;

static double cc_f(double s, const void* vc)
{
    const cc_ctx* c = (const cc_ctx*)vc;
    return ora_point_cell(c->p, c->q, s, c->a2, c->b2, c->ell);
}

double ora_cell_cell(int p, int q, double a, double b, double a2, double b2, double ell)
{
    cc_ctx c = {p, q, a2, b2, ell};
    return integrate(cc_f, &c, a, b, REL_OUTER);
}

/* Generic integral of d^m k(r) over [a,b] in r (used to pin the rule). */
typedef struct { int m; double ell; } r_ctx;
static double r_f(double r, const void* vc)
{
    const r_ctx* c = (const r_ctx*)vc;
    return ora_kder(c->m, r, c->ell);
}
double ora_integrate_kder(int m, double a, double b, double ell)
{
    r_ctx c = {m, ell};
    return integrate(r_f, &c, a, b, 1e-14);
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
void ora_cell_cell_matrix(int p, int q, int n1, const double* e1, int n2,
                          const double* e2, double ell, double* out)
{
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n2; ++j)
            out[(size_t)i * n2 + j] = ora_cell_cell(p, q, e1[i], e1[i + 1], e2[j], e2[j + 1], ell);
}

/* out[i*n2 + j] = Q^{pq}(x[i], [e2[j],e2[j+1]]) */
void ora_point_cell_matrix(int p, int q, int n1, const double* x, int n2,
                           const double* e2, double ell, double* out)
{
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n2; ++j)
            out[(size_t)i * n2 + j] = ora_point_cell(p, q, x[i], e2[j], e2[j + 1], ell);
}

/* out[i*n2 + j] = P^{pq}(x[i], x2[j]) */
void ora_point_point_matrix(int p, int q, int n1, const double* x, int n2,
                            const double* x2, double ell, double* out)
{
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n2; ++j)
            out[(size_t)i * n2 + j] = ora_point_point(p, q, x[i], x2[j], ell);
}
