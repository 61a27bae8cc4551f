/*
 * scpic_oracle.c -- plain, slow, FP64 CPU oracle of the 2D particle-in-cell
 * space-charge step (push -> charge deposit -> open-boundary Poisson solve ->
 * field -> gather and kick).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: it exists so that the tests, the smoke check and the CPU
 * baseline leg of the benchmark have an independent answer to compare the HIP
 * path against.  It shares no code, header, table or constant generator with
 * the HIP library.
 *
 * Build:  gcc -O2 -std=c11 -fopenmp -ffp-contract=off -fno-fast-math -fPIC -shared
 * (-ffp-contract=off: every expression below is evaluated as written, each
 *  operation correctly rounded, no fused multiply-add.)
 *
 * Conventions (shared by the tests):
 *   particles   structure of arrays x, px, y, py (m, rad); lost[p] != 0 means
 *               the particle has left the grid and is frozen.  Lattices with
 *               thick elements also carry sigma = s - c beta0 t (m) and its
 *               conjugate p_sigma (Sec. III); other elements leave them alone.
 *   grid        nx, ny nodes at x_min + i*dx, y_min + j*dy; node arrays are
 *               row-major [i*ny + j] (i along x).
 *   elements    kind[e], par[e*16 + k]:
 *                 1 LIN2X2   par[0..3] x-block, par[4..7] y-block (row-major)
 *                 2 LIN4X4   par[0..15] row-major on (x, px, y, py)
 *                 3 SEXTUPOLE_THIN  par[0] = k2*L
 *                 4 SPACE_CHARGE    par[0] = kick coefficient kappa
 *                 5 QUAD_THICK      par[0] = k1 (1/m^2), par[1] = L (m),
 *                                   par[2] = 1/gamma0^2
 *                 6 SEXT_THICK      par[0] = k2 (1/m^3), par[1] = L (m),
 *                                   par[2] = 1/gamma0^2, par[3] = steps n >= 1
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_LIN2X2 1
#define ORC_LIN4X4 2
#define ORC_SEXT_THIN 3
#define ORC_SC 4
#define ORC_QUAD_THICK 5
#define ORC_SEXT_THICK 6

/* Fixed-point charge assignment: 12 fractional bits per axis, so the four
 * weights of one particle sum to exactly 2^24 charge units. */
#define ORC_FRAC_ONE 4096
#define ORC_CHARGE_ONE 16777216.0 /* 2^24 */

typedef struct {
    int nx, ny;
    double x_min, y_min, dx, dy;
    double inv_dx, inv_dy;
} orc_grid;

static orc_grid make_grid(int nx, int ny, double x_min, double y_min, double dx, double dy)
{
    orc_grid g;
    g.nx = nx;
    g.ny = ny;
    g.x_min = x_min;
    g.y_min = y_min;
    g.dx = dx;
    g.dy = dy;
    g.inv_dx = 1.0 / dx;
    g.inv_dy = 1.0 / dy;
    return g;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel regions (n >= 1); returns the count in
 * effect afterwards.  Timing only: results do not depend on it. */
int orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
    return orc_num_threads();
}

/* ------------------------------------------------------------------------ */
/* Single-particle mechanics (Sec. III): each element is a symplectic map.   */
/* ------------------------------------------------------------------------ */

/* One element applied to one particle.  A linear element multiplies the
 * phase-space vector by its transfer matrix (v <- M v).  The thin sextupole is
 * the kick step of the split thick-sextupole integrator of Sec. III-C with the
 * drift parts removed: with V = k2 (x^3 - 3 x y^2) / 6 and integrated strength
 * k2*L, the momenta change by -dV/dx * L and -dV/dy * L. */
static void push_linear(double v[6], int kind, const double *m)
{
    double X = v[0], PX = v[1], Y = v[2], PY = v[3];
    if (kind == ORC_LIN2X2) {
        v[0] = m[0] * X + m[1] * PX;
        v[1] = m[2] * X + m[3] * PX;
        v[2] = m[4] * Y + m[5] * PY;
        v[3] = m[6] * Y + m[7] * PY;
    } else if (kind == ORC_LIN4X4) {
        v[0] = m[0] * X + m[1] * PX + m[2] * Y + m[3] * PY;
        v[1] = m[4] * X + m[5] * PX + m[6] * Y + m[7] * PY;
        v[2] = m[8] * X + m[9] * PX + m[10] * Y + m[11] * PY;
        v[3] = m[12] * X + m[13] * PX + m[14] * Y + m[15] * PY;
    } else if (kind == ORC_SEXT_THIN) {
        double k2l = m[0];
        v[1] = PX - 0.5 * k2l * (X * X - Y * Y);
        v[3] = PY + k2l * X * Y;
    }
}

/* One transverse plane of the thick quadrupole (Sec. III-B), the exact flow of
 * H_approx (eq. H, h = 0, e A_s / p0 = -k1 (x^2 - y^2) / 2) over length L:
 * with q = 1 - p_sigma the plane obeys u' = q p_u, p_u' = -K u, where K = k1
 * for x and K = -k1 for y.  A focusing plane (K > 0) turns by the angle
 * sqrt(K q) L:
 *   u(L)   = u cos + sqrt(q/K) p_u sin,    p_u(L) = p_u cos - sqrt(K/q) u sin;
 * a defocusing plane takes cosh and sinh, with the sign of the second p_u term
 * flipped; K = 0 is the drift u(L) = u + q p_u L.  Returns the integral of
 * p_u(s)^2 over the element, which the path-length equation needs: writing
 * p_u(s) = A c(s) + B s(s) with the plane's pair of functions,
 *   focusing    A^2 (L/2 + sin(2 phi)/(4 w)) + A B sin(phi)^2 / w
 *               + B^2 (L/2 - sin(2 phi)/(4 w)),
 *   defocusing  A^2 (L/2 + sinh(2 phi)/(4 w)) + A B sinh(phi)^2 / w
 *               + B^2 (sinh(2 phi)/(4 w) - L/2),
 * where w = sqrt(|K| q) and phi = w L. */
static double quad_plane(double *u, double *pu, double K, double q, double L)
{
    double u0 = *u, p0 = *pu;
    if (K == 0.0) {
        *u = u0 + q * p0 * L;
        return p0 * p0 * L;
    }
    double k = fabs(K);
    double w = sqrt(k * q);
    double phi = w * L;
    double A = p0, B;
    if (K > 0.0) {
        double c = cos(phi), s = sin(phi);
        *u = u0 * c + sqrt(q / k) * p0 * s;
        *pu = p0 * c - sqrt(k / q) * u0 * s;
        B = -sqrt(k / q) * u0;
        double s2 = sin(2.0 * phi) / (4.0 * w);
        return A * A * (0.5 * L + s2) + A * B * s * s / w + B * B * (0.5 * L - s2);
    }
    double c = cosh(phi), s = sinh(phi);
    *u = u0 * c + sqrt(q / k) * p0 * s;
    *pu = p0 * c + sqrt(k / q) * u0 * s;
    B = sqrt(k / q) * u0;
    double s2 = sinh(2.0 * phi) / (4.0 * w);
    return A * A * (0.5 * L + s2) + A * B * s * s / w + B * B * (s2 - 0.5 * L);
}

/* Thick quadrupole with chromatic focusing (Sec. III-B): both planes as above
 * with q = 1 - p_sigma; p_sigma is constant and
 *   sigma(L) = sigma(0) + p_sigma L / gamma0^2 - (1/2) int_0^L (px^2 + py^2) ds. */
static void push_quad_thick(double v[6], const double *m)
{
    double k1 = m[0], L = m[1], ig2 = m[2];
    double q = 1.0 - v[5];
    double ix = quad_plane(&v[0], &v[1], k1, q, L);
    double iy = quad_plane(&v[2], &v[3], -k1, q, L);
    v[4] = v[4] + v[5] * L * ig2 - 0.5 * (ix + iy);
}

/* Exact flow of H0 = (px^2 + py^2)/2 + p_sigma^2/(2 gamma0^2)
 *                   - (px^2 + py^2) p_sigma / 2      (Sec. III-C)
 * over length t: the momenta are constant, dx/ds = px (1 - p_sigma),
 * dy/ds = py (1 - p_sigma), dsigma/ds = p_sigma/gamma0^2 - (px^2 + py^2)/2. */
static void flow_h0(double v[6], double t, double ig2)
{
    double q = 1.0 - v[5];
    v[0] = v[0] + v[1] * q * t;
    v[2] = v[2] + v[3] * q * t;
    v[4] = v[4] + (v[5] * ig2 - 0.5 * (v[1] * v[1] + v[3] * v[3])) * t;
}

/* Exact flow of V = k2 (x^3 - 3 x y^2) / 6 over length t: positions fixed,
 * px -= dV/dx t = (k2/2)(x^2 - y^2) t,  py -= dV/dy t = -k2 x y t. */
static void flow_v(double v[6], double t, double k2)
{
    double X = v[0], Y = v[2];
    v[1] = v[1] - 0.5 * k2 * (X * X - Y * Y) * t;
    v[3] = v[3] + k2 * X * Y * t;
}

/* Thick sextupole (Sec. III-C, eq. Sym2): H_approx = H0 + V is advanced by the
 * symmetric product of exact flows
 *   H0 over a h, V over b h, H0 over c h, V over b h, H0 over a h
 * with a = (1 - 1/sqrt 3)/2, b = 1/2, c = 1/sqrt 3, applied n times with
 * h = L / n (n = 1 is one product over the whole element). */
static void push_sext_thick(double v[6], const double *m)
{
    double k2 = m[0], L = m[1], ig2 = m[2];
    int n = (int)m[3];
    double h = L / (double)n;
    double c = 1.0 / sqrt(3.0);
    double a = 0.5 * (1.0 - c), b = 0.5;
    for (int i = 0; i < n; ++i) {
        flow_h0(v, a * h, ig2);
        flow_v(v, b * h, k2);
        flow_h0(v, c * h, ig2);
        flow_v(v, b * h, k2);
        flow_h0(v, a * h, ig2);
    }
}

static int is_thick(int kind) { return kind == ORC_QUAD_THICK || kind == ORC_SEXT_THICK; }

/* Apply the non-space-charge elements in order; lost particles are frozen.
 * sigma and psigma may be NULL when no element is thick; returns -1 (and
 * moves nothing) when a thick element meets NULL longitudinal arrays or a
 * thick sextupole has n < 1 steps. */
int orc_push(int64_t n, double *x, double *px, double *y, double *py, double *sigma,
             double *psigma, const uint8_t *lost, int n_el, const int32_t *kind, const double *par)
{
    for (int e = 0; e < n_el; ++e) {
        if (is_thick(kind[e]) && (!sigma || !psigma)) return -1;
        if (kind[e] == ORC_SEXT_THICK && par[16 * e + 3] < 1.0) return -1;
    }
    int64_t p;
#pragma omp parallel for schedule(static)
    for (p = 0; p < n; ++p) {
        if (lost && lost[p]) continue;
        double v[6] = {x[p], px[p], y[p], py[p], sigma ? sigma[p] : 0.0, psigma ? psigma[p] : 0.0};
        for (int e = 0; e < n_el; ++e) {
            const double *m = par + 16 * e;
            if (kind[e] == ORC_QUAD_THICK)
                push_quad_thick(v, m);
            else if (kind[e] == ORC_SEXT_THICK)
                push_sext_thick(v, m);
            else if (kind[e] != ORC_SC)
                push_linear(v, kind[e], m);
        }
        x[p] = v[0];
        px[p] = v[1];
        y[p] = v[2];
        py[p] = v[3];
        if (sigma) sigma[p] = v[4];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Charge assignment (Sec. IV-A): cloud-in-cell onto the four nodes of the   */
/* cell holding the particle, weights bilinear in the position inside it.   */
/* ------------------------------------------------------------------------ */

/* Cell index and the integer weights of one particle; returns 0 when the
 * particle is outside the half-open domain [x_min, x_min + (nx-1) dx) x [...]
 * (a NaN coordinate is outside).  w[0..3] are the weights of nodes (i,j),
 * (i+1,j), (i,j+1), (i+1,j+1); they are the paper's bilinear fractions rounded
 * to 12 bits per axis and sum to exactly 2^24. */
static int cic_weights(const orc_grid *g, double x, double y, int *ci, int *cj, int64_t w[4])
{
    double tx = (x - g->x_min) * g->inv_dx;
    double ty = (y - g->y_min) * g->inv_dy;
    if (!(tx >= 0.0 && tx < (double)(g->nx - 1))) return 0;
    if (!(ty >= 0.0 && ty < (double)(g->ny - 1))) return 0;
    double fi = floor(tx), fj = floor(ty);
    double fx = tx - fi, fy = ty - fj; /* exact */
    int64_t a = (int64_t)floor(fx * 4096.0 + 0.5);
    int64_t b = (int64_t)floor(fy * 4096.0 + 0.5);
    *ci = (int)fi;
    *cj = (int)fj;
    w[0] = (ORC_FRAC_ONE - a) * (ORC_FRAC_ONE - b);
    w[1] = a * (ORC_FRAC_ONE - b);
    w[2] = (ORC_FRAC_ONE - a) * b;
    w[3] = a * b;
    return 1;
}

/* Deposit all alive particles into q (int64 charge units, overwritten).
 * Particles outside the domain are marked lost.  Returns the number of
 * particles deposited. */
int64_t orc_deposit(int64_t n, const double *x, const double *y, uint8_t *lost, int nx, int ny,
                    double x_min, double y_min, double dx, double dy, int64_t *q)
{
    orc_grid g = make_grid(nx, ny, x_min, y_min, dx, dy);
    int64_t cells = (int64_t)nx * ny;
    int nt = orc_num_threads();
    int64_t *priv = (int64_t *)calloc((size_t)(nt * cells), sizeof(int64_t));
    int64_t n_in = 0;
    if (!priv) return -1;
#pragma omp parallel reduction(+ : n_in)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        int64_t *mine = priv + (int64_t)t * cells;
        int64_t p;
#pragma omp for schedule(static)
        for (p = 0; p < n; ++p) {
            if (lost && lost[p]) continue;
            int i, j;
            int64_t w[4];
            if (!cic_weights(&g, x[p], y[p], &i, &j, w)) {
                if (lost) lost[p] = 1;
                continue;
            }
            mine[(int64_t)i * ny + j] += w[0];
            mine[(int64_t)(i + 1) * ny + j] += w[1];
            mine[(int64_t)i * ny + j + 1] += w[2];
            mine[(int64_t)(i + 1) * ny + j + 1] += w[3];
            n_in += 1;
        }
    }
    for (int64_t c = 0; c < cells; ++c) {
        int64_t s = 0;
        for (int t = 0; t < nt; ++t) s += priv[(int64_t)t * cells + c];
        q[c] = s;
    }
    free(priv);
    return n_in;
}

/* ------------------------------------------------------------------------ */
/* Open-boundary Poisson solve (Hockney's free-space Green's function).      */
/* ------------------------------------------------------------------------ */

/* Antiderivative of ln(x^2 + y^2) in both variables (d2F/dxdy = ln(x^2+y^2)),
 * for x, y > 0. */
static double log_antiderivative(double x, double y)
{
    return x * y * (log(x * x + y * y) - 3.0) + x * x * atan(y / x) + y * y * atan(x / y);
}

/* Green's function of the 2D Laplacian normalised so that lap G = -2 pi delta:
 * G(X, Y) = -ln(r) = -ln(X^2 + Y^2) / 2 at offsets (di*dx, dj*dy) != 0; at the
 * origin the singular value is replaced by its average over one cell. */
double orc_green(int di, int dj, double dx, double dy)
{
    if (di == 0 && dj == 0) {
        double a = 0.5 * dx, b = 0.5 * dy;
        return -log_antiderivative(a, b) / (2.0 * a * b);
    }
    double X = di * dx, Y = dj * dy;
    return -0.5 * log(X * X + Y * Y);
}

/* Potential phi = G (*) rho by the direct sum over all charged nodes, at the
 * nodes i = -1..nx, j = -1..ny (one ring of nodes around the grid, needed by
 * the centred differences of the field).  rho = q * scale.
 * phi is (nx+2) x (ny+2), row-major, phi[(i+1)*(ny+2) + (j+1)].
 * The sum is accumulated in extended precision (long double): the field is a
 * difference of neighbouring potentials two orders of magnitude smaller than
 * the potentials themselves, so FP64 accumulation of thousands of terms would
 * leave the oracle's own rounding near 1e-12 of the field on fine grids. */
void orc_potential(const int64_t *q, double scale, int nx, int ny, double dx, double dy, double *phi)
{
    /* G depends only on |di|, |dj| <= nx, ny: tabulate it once. */
    int gx = nx + 1, gy = ny + 1;
    double *G = (double *)malloc(sizeof(double) * (size_t)gx * gy);
    for (int di = 0; di < gx; ++di)
        for (int dj = 0; dj < gy; ++dj) G[di * gy + dj] = orc_green(di, dj, dx, dy);
    int64_t ti;
    int64_t targets = (int64_t)(nx + 2) * (ny + 2);
#pragma omp parallel for schedule(dynamic, 16)
    for (ti = 0; ti < targets; ++ti) {
        int i = (int)(ti / (ny + 2)) - 1;
        int j = (int)(ti % (ny + 2)) - 1;
        long double s = 0.0L;
        for (int k = 0; k < nx; ++k)
            for (int l = 0; l < ny; ++l) {
                int64_t c = q[(int64_t)k * ny + l];
                if (c == 0) continue;
                s += (long double)G[abs(i - k) * gy + abs(j - l)] * ((long double)c * scale);
            }
        phi[ti] = (double)s;
    }
    free(G);
}

/* ------------------------------------------------------------------------ */
/* Grounded rectangular pipe (Sec. IV-B): the 5-point discrete Poisson       */
/* equation with u = 0 on the walls.                                          */
/* ------------------------------------------------------------------------ */

/* Potential in a grounded rectangular pipe whose walls pass through node 0
 * and node nx along x (node nx is one spacing past the last grid node), and
 * through node 0 and node ny along y.  phi solves, at every interior node
 * (1 <= i <= nx-1, 1 <= j <= ny-1),
 *   (phi[i-1][j] - 2 phi[i][j] + phi[i+1][j]) / dx^2
 *     + (phi[i][j-1] - 2 phi[i][j] + phi[i][j+1]) / dy^2 = -2 pi rho[i][j] / (dx dy),
 * with phi = 0 on the walls (the charge of the wall nodes i = 0 or j = 0 is
 * taken by the grounded wall) -- the same normalisation as the open-boundary
 * solve (lap G = -2 pi delta per unit charge).  The solution is written out as
 * its expansion in the eigenvectors sin(p pi i / nx) sin(q pi j / ny) of the
 * discrete Laplacian (eigenvalue -4 (sin^2(p pi/(2 nx))/dx^2 +
 * sin^2(q pi/(2 ny))/dy^2)), summed separably in long double.  Output layout
 * as orc_potential: nodes -1..nx by -1..ny, with the walls 0 and node -1 the
 * mirror image -phi[1] (the odd extension across the wall at node 0). */
void orc_potential_pipe(const int64_t *q, double scale, int nx, int ny, double dx, double dy,
                        double *phi)
{
    const long double pi = 3.141592653589793238462643383279502884L;
    int mi = nx - 1, mj = ny - 1; /* interior nodes per axis */
    long double *sx = (long double *)malloc(sizeof(long double) * (size_t)nx * nx);
    long double *sy = (long double *)malloc(sizeof(long double) * (size_t)ny * ny);
    long double *a = (long double *)calloc((size_t)nx * ny, sizeof(long double));
    long double *b = (long double *)calloc((size_t)nx * ny, sizeof(long double));
    for (int p = 0; p < nx; ++p)
        for (int i = 0; i < nx; ++i) sx[p * nx + i] = sinl(pi * p * i / nx);
    for (int r = 0; r < ny; ++r)
        for (int j = 0; j < ny; ++j) sy[r * ny + j] = sinl(pi * r * j / ny);
    /* forward: f_hat[p][r] = sum_ij f[i][j] sin(p pi i/nx) sin(r pi j/ny) */
    for (int i = 1; i <= mi; ++i)
        for (int r = 1; r <= mj; ++r) {
            long double s = 0.0L;
            for (int j = 1; j <= mj; ++j) {
                long double f = -2.0L * pi * ((long double)q[(int64_t)i * ny + j] * scale) /
                                ((long double)dx * dy);
                s += f * sy[r * ny + j];
            }
            a[i * ny + r] = s;
        }
    for (int p = 1; p <= mi; ++p)
        for (int r = 1; r <= mj; ++r) {
            long double s = 0.0L;
            for (int i = 1; i <= mi; ++i) s += a[i * ny + r] * sx[p * nx + i];
            long double spx = sinl(pi * p / (2.0L * nx)), spy = sinl(pi * r / (2.0L * ny));
            long double lam = -4.0L * (spx * spx / ((long double)dx * dx) +
                                       spy * spy / ((long double)dy * dy));
            b[p * ny + r] = s / lam;
        }
    /* inverse: phi[i][j] = (2/nx)(2/ny) sum_pr phi_hat[p][r] sin(..) sin(..) */
    for (int p = 1; p <= mi; ++p)
        for (int j = 1; j <= mj; ++j) {
            long double s = 0.0L;
            for (int r = 1; r <= mj; ++r) s += b[p * ny + r] * sy[r * ny + j];
            a[p * ny + j] = s;
        }
    int sy2 = ny + 2;
    memset(phi, 0, sizeof(double) * (size_t)(nx + 2) * sy2);
    for (int i = 1; i <= mi; ++i)
        for (int j = 1; j <= mj; ++j) {
            long double s = 0.0L;
            for (int p = 1; p <= mi; ++p) s += a[p * ny + j] * sx[p * nx + i];
            phi[(i + 1) * sy2 + (j + 1)] = (double)(s * 4.0L / ((long double)nx * ny));
        }
    /* odd images across the walls at node 0: node -1 mirrors node 1 */
    for (int j = 0; j < ny + 2; ++j) phi[0 * sy2 + j] = -phi[2 * sy2 + j];
    for (int i = 0; i < nx + 2; ++i) phi[i * sy2 + 0] = -phi[i * sy2 + 2];
    free(sx);
    free(sy);
    free(a);
    free(b);
}

/* E = -grad(phi) by centred differences at the nodes 0..nx-1, 0..ny-1. */
void orc_field(const double *phi, int nx, int ny, double dx, double dy, double *ex, double *ey)
{
    int sy = ny + 2;
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
            double pxp = phi[(i + 2) * sy + (j + 1)], pxm = phi[i * sy + (j + 1)];
            double pyp = phi[(i + 1) * sy + (j + 2)], pym = phi[(i + 1) * sy + j];
            ex[i * ny + j] = -(pxp - pxm) / (2.0 * dx);
            ey[i * ny + j] = -(pyp - pym) / (2.0 * dy);
        }
}

/* Interpolate the node field to each alive particle with the same four
 * weights as the deposit and kick its momenta: p += kappa * w_p * E, with the
 * particle's weight w_p = wt[p] (1 when wt is NULL).  A particle outside the domain is
 * marked lost instead.  (Sec. IV: the transverse kick is proportional to the
 * line density at the particle times the field of the transverse
 * distribution times the distance since the previous space-charge location;
 * kappa carries that length and the perveance, w_p the line density relative
 * to its peak.) */
void orc_kick(int64_t n, const double *x, double *px, const double *y, double *py, uint8_t *lost,
              const float *wt, int nx, int ny, double x_min, double y_min, double dx, double dy,
              const double *ex, const double *ey, double kappa)
{
    orc_grid g = make_grid(nx, ny, x_min, y_min, dx, dy);
    int64_t p;
#pragma omp parallel for schedule(static)
    for (p = 0; p < n; ++p) {
        if (lost && lost[p]) continue;
        int i, j;
        int64_t w[4];
        if (!cic_weights(&g, x[p], y[p], &i, &j, w)) {
            if (lost) lost[p] = 1;
            continue;
        }
        int64_t c00 = (int64_t)i * ny + j, c10 = c00 + ny, c01 = c00 + 1, c11 = c00 + ny + 1;
        double exp_ = ((double)w[0] * ex[c00] + (double)w[1] * ex[c10] + (double)w[2] * ex[c01] +
                       (double)w[3] * ex[c11]) / ORC_CHARGE_ONE;
        double eyp = ((double)w[0] * ey[c00] + (double)w[1] * ey[c10] + (double)w[2] * ey[c01] +
                      (double)w[3] * ey[c11]) / ORC_CHARGE_ONE;
        double k = wt ? kappa * (double)wt[p] : kappa;
        px[p] += k * exp_;
        py[p] += k * eyp;
    }
}

/* ------------------------------------------------------------------------ */
/* Potential interpolation (Sec. IV-C): the bicubic surface through the 4x4  */
/* nodes around the particle's cell, field as its analytic gradient.         */
/* ------------------------------------------------------------------------ */

/* Uniform cubic B-spline basis on the cell fraction t in [0, 1): the weights
 * of nodes i-1, i, i+1, i+2 and their derivatives in t. */
static void bspline3(double t, double b[4], double db[4])
{
    double u = 1.0 - t;
    b[0] = u * u * u / 6.0;
    b[1] = (3.0 * t * t * t - 6.0 * t * t + 4.0) / 6.0;
    b[2] = (-3.0 * t * t * t + 3.0 * t * t + 3.0 * t + 1.0) / 6.0;
    b[3] = t * t * t / 6.0;
    db[0] = -u * u / 2.0;
    db[1] = (3.0 * t * t - 4.0 * t) / 2.0;
    db[2] = (-3.0 * t * t + 2.0 * t + 1.0) / 2.0;
    db[3] = t * t / 2.0;
}

/* Potential and field at (x, y) from the node potential phi ((nx+2)(ny+2),
 * nodes -1..nx by -1..ny as orc_potential writes it):
 *   u = sum_{m,n} phi[i+m-1][j+n-1] B_m(tx) B_n(ty),  E = -grad u,
 * with i = floor(tx), tx = (x - x_min)/dx (and likewise in y).  Returns 0
 * outside the half-open domain of the charge assignment. */
static int bspline_field(const orc_grid *g, const double *phi, double x, double y, double *u,
                         double *ex, double *ey)
{
    double tx = (x - g->x_min) * g->inv_dx;
    double ty = (y - g->y_min) * g->inv_dy;
    if (!(tx >= 0.0 && tx < (double)(g->nx - 1))) return 0;
    if (!(ty >= 0.0 && ty < (double)(g->ny - 1))) return 0;
    int i = (int)floor(tx), j = (int)floor(ty);
    double bx[4], dbx[4], by[4], dby[4];
    bspline3(tx - i, bx, dbx);
    bspline3(ty - j, by, dby);
    int64_t s = g->ny + 2;
    double su = 0.0, sx = 0.0, sy = 0.0;
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) {
            /* node (i+m-1, j+n-1) sits at row i+m, column j+n of phi */
            double v = phi[(int64_t)(i + m) * s + (j + n)];
            su += v * bx[m] * by[n];
            sx += v * dbx[m] * by[n];
            sy += v * bx[m] * dby[n];
        }
    *u = su;
    *ex = -sx * g->inv_dx;
    *ey = -sy * g->inv_dy;
    return 1;
}

/* Evaluate the interpolated potential and field at n points (for the pins);
 * points outside the domain get NaN. */
void orc_bspline_eval(int64_t n, const double *x, const double *y, const double *phi, int nx,
                      int ny, double x_min, double y_min, double dx, double dy, double *u,
                      double *ex, double *ey)
{
    orc_grid g = make_grid(nx, ny, x_min, y_min, dx, dy);
    for (int64_t p = 0; p < n; ++p)
        if (!bspline_field(&g, phi, x[p], y[p], &u[p], &ex[p], &ey[p])) u[p] = ex[p] = ey[p] = NAN;
}

/* Kick with the interpolated field: p += kappa w_p E(x, y), E from the
 * B-spline surface of the node potential. */
void orc_kick_bspline(int64_t n, const double *x, double *px, const double *y, double *py,
                      uint8_t *lost, const float *wt, int nx, int ny, double x_min, double y_min,
                      double dx, double dy, const double *phi, double kappa)
{
    orc_grid g = make_grid(nx, ny, x_min, y_min, dx, dy);
    int64_t p;
#pragma omp parallel for schedule(static)
    for (p = 0; p < n; ++p) {
        if (lost && lost[p]) continue;
        double u, ex, ey;
        if (!bspline_field(&g, phi, x[p], y[p], &u, &ex, &ey)) {
            if (lost) lost[p] = 1;
            continue;
        }
        double k = wt ? kappa * (double)wt[p] : kappa;
        px[p] += k * ex;
        py[p] += k * ey;
    }
}

/* The whole space-charge step at one location: deposit, potential (open
 * boundary, or the grounded pipe when pipe != 0), field, kick.  scale converts charge units to the normalised density (1/(2^24 N0)
 * for N0 initial macro-particles, so the total charge is 1).  ex/ey, when not
 * NULL, receive the node field.  Returns the number of particles deposited. */
static int64_t space_charge_step(int64_t n, double *x, double *px, double *y, double *py,
                                 uint8_t *lost, const float *wt, int nx, int ny, double x_min,
                                 double y_min, double dx, double dy, double scale, double kappa,
                                 double *ex_out, double *ey_out, int pipe, int bspline);

int64_t orc_space_charge(int64_t n, double *x, double *px, double *y, double *py, uint8_t *lost,
                         const float *wt, int nx, int ny, double x_min, double y_min, double dx,
                         double dy, double scale, double kappa, double *ex_out, double *ey_out,
                         int pipe)
{
    return space_charge_step(n, x, px, y, py, lost, wt, nx, ny, x_min, y_min, dx, dy, scale, kappa,
                             ex_out, ey_out, pipe, 0);
}

/* As orc_space_charge, with the kick's field from the B-spline surface of the
 * potential (Sec. IV-C) instead of the cloud-in-cell gather of node fields. */
int64_t orc_space_charge_bspline(int64_t n, double *x, double *px, double *y, double *py,
                                 uint8_t *lost, const float *wt, int nx, int ny, double x_min,
                                 double y_min, double dx, double dy, double scale, double kappa,
                                 int pipe)
{
    return space_charge_step(n, x, px, y, py, lost, wt, nx, ny, x_min, y_min, dx, dy, scale, kappa,
                             NULL, NULL, pipe, 1);
}

static int64_t space_charge_step(int64_t n, double *x, double *px, double *y, double *py,
                                 uint8_t *lost, const float *wt, int nx, int ny, double x_min,
                                 double y_min, double dx, double dy, double scale, double kappa,
                                 double *ex_out, double *ey_out, int pipe, int bspline)
{
    int64_t cells = (int64_t)nx * ny;
    int64_t *q = (int64_t *)malloc(sizeof(int64_t) * (size_t)cells);
    double *phi = (double *)malloc(sizeof(double) * (size_t)(nx + 2) * (ny + 2));
    double *ex = ex_out ? ex_out : (double *)malloc(sizeof(double) * (size_t)cells);
    double *ey = ey_out ? ey_out : (double *)malloc(sizeof(double) * (size_t)cells);
    int64_t n_in = orc_deposit(n, x, y, lost, nx, ny, x_min, y_min, dx, dy, q);
    if (pipe)
        orc_potential_pipe(q, scale, nx, ny, dx, dy, phi);
    else
        orc_potential(q, scale, nx, ny, dx, dy, phi);
    orc_field(phi, nx, ny, dx, dy, ex, ey);
    if (bspline)
        orc_kick_bspline(n, x, px, y, py, lost, wt, nx, ny, x_min, y_min, dx, dy, phi, kappa);
    else
        orc_kick(n, x, px, y, py, lost, wt, nx, ny, x_min, y_min, dx, dy, ex, ey, kappa);
    if (!ex_out) free(ex);
    if (!ey_out) free(ey);
    free(phi);
    free(q);
    return n_in;
}

/* ------------------------------------------------------------------------ */
/* Longitudinal space charge of a long bunch (Sec. IV): the line density     */
/* lambda(sigma) from a histogram of sigma, the transverse kick scaled by     */
/* lambda / lambda_peak and the longitudinal kick from the potential.        */
/* ------------------------------------------------------------------------ */

/* Node k and the two fixed-point weights of sigma on the line of nz nodes
 * z_min + k dz: t = (s - z_min)(1/dz), k = floor(t), a = floor((t - k) 4096 + 0.5),
 * weights 4096 - a at node k and a at node k + 1 (the one-dimensional form of
 * the transverse assignment).  Returns 0 outside [z_min, z_min + (nz-1) dz). */
static int line_weights(double s, int nz, double z_min, double inv_dz, int *k, int64_t w[2])
{
    double t = (s - z_min) * inv_dz;
    if (!(t >= 0.0 && t < (double)(nz - 1))) return 0;
    double fk = floor(t);
    int64_t a = (int64_t)floor((t - fk) * 4096.0 + 0.5);
    *k = (int)fk;
    w[0] = ORC_FRAC_ONE - a;
    w[1] = a;
    return 1;
}

/* Transverse charge q (as orc_deposit, nx*ny) and line-density histogram h
 * (nz nodes, 4096 units per particle) of the particles inside both domains;
 * a particle outside either is marked lost and deposits nothing.  Returns the
 * number deposited. */
int64_t orc_deposit_line(int64_t n, const double *x, const double *y, const double *sigma,
                         uint8_t *lost, int nx, int ny, double x_min, double y_min, double dx,
                         double dy, int nz, double z_min, double dz, int64_t *q, int64_t *h)
{
    orc_grid g = make_grid(nx, ny, x_min, y_min, dx, dy);
    double inv_dz = 1.0 / dz;
    memset(q, 0, sizeof(int64_t) * (size_t)nx * ny);
    memset(h, 0, sizeof(int64_t) * (size_t)nz);
    int64_t n_in = 0;
    for (int64_t p = 0; p < n; ++p) {
        if (lost && lost[p]) continue;
        int i, j, k;
        int64_t w[4], wl[2];
        if (!cic_weights(&g, x[p], y[p], &i, &j, w) ||
            !line_weights(sigma[p], nz, z_min, inv_dz, &k, wl)) {
            if (lost) lost[p] = 1;
            continue;
        }
        q[(int64_t)i * ny + j] += w[0];
        q[(int64_t)(i + 1) * ny + j] += w[1];
        q[(int64_t)i * ny + j + 1] += w[2];
        q[(int64_t)(i + 1) * ny + j + 1] += w[3];
        h[k] += wl[0];
        h[k + 1] += wl[1];
        n_in += 1;
    }
    return n_in;
}

/* Line-density factors at the nodes, relative to the peak:
 *   lw[k] = h[k] / max h,   ld[k] = (h[k+1] - h[k-1]) / (2 dz max h)
 * (centred difference, h = 0 beyond the line; all zero for an empty line). */
void orc_line_table(const int64_t *h, int nz, double dz, double *lw, double *ld)
{
    int64_t hmax = 0;
    for (int k = 0; k < nz; ++k)
        if (h[k] > hmax) hmax = h[k];
    for (int k = 0; k < nz; ++k) {
        if (hmax == 0) {
            lw[k] = 0.0;
            ld[k] = 0.0;
            continue;
        }
        int64_t up = k + 1 < nz ? h[k + 1] : 0, down = k > 0 ? h[k - 1] : 0;
        lw[k] = (double)h[k] / (double)hmax;
        ld[k] = (double)(up - down) / (2.0 * dz * (double)hmax);
    }
}

/* One space-charge step of a long bunch in the grounded rectangular pipe
 * (Sec. IV with the solver of Sec. IV-B): deposit (transverse charge and line
 * density), pipe potential phi and field E, then for every particle, with
 * w = lambda(sigma)/lambda_peak and d = lambda'(sigma)/lambda_peak
 * interpolated from the node factors with its line weights, and phi, E
 * interpolated with its transverse weights:
 *   px += kappa w Ex,  py += kappa w Ey,  p_sigma -= gamma0 kappa phi d.
 * The longitudinal kick's coefficient e/(m gamma0^2 beta0^2 c^2) is gamma0
 * times the transverse one, e/(m gamma0^3 beta0^2 c^2), which kappa carries.
 * lw_out, ld_out (nz) and phi_out ((nx+2)(ny+2), as orc_potential_pipe)
 * receive the tables when not NULL.  Returns the number deposited, -1 when out
 * of memory. */
int64_t orc_space_charge_line(int64_t n, double *x, double *px, double *y, double *py,
                              const double *sigma, double *psigma, uint8_t *lost, int nx, int ny,
                              double x_min, double y_min, double dx, double dy, int nz,
                              double z_min, double dz, double gamma0, double scale, double kappa,
                              double *lw_out, double *ld_out, double *phi_out)
{
    int64_t cells = (int64_t)nx * ny;
    int64_t *q = (int64_t *)malloc(sizeof(int64_t) * (size_t)cells);
    int64_t *h = (int64_t *)malloc(sizeof(int64_t) * (size_t)nz);
    double *phi = (double *)malloc(sizeof(double) * (size_t)(nx + 2) * (ny + 2));
    double *ex = (double *)malloc(sizeof(double) * (size_t)cells);
    double *ey = (double *)malloc(sizeof(double) * (size_t)cells);
    double *lw = (double *)malloc(sizeof(double) * (size_t)nz);
    double *ld = (double *)malloc(sizeof(double) * (size_t)nz);
    int64_t n_in = -1;
    if (!q || !h || !phi || !ex || !ey || !lw || !ld) goto done;
    n_in = orc_deposit_line(n, x, y, sigma, lost, nx, ny, x_min, y_min, dx, dy, nz, z_min, dz, q,
                            h);
    orc_potential_pipe(q, scale, nx, ny, dx, dy, phi);
    orc_field(phi, nx, ny, dx, dy, ex, ey);
    orc_line_table(h, nz, dz, lw, ld);
    {
        orc_grid g = make_grid(nx, ny, x_min, y_min, dx, dy);
        double inv_dz = 1.0 / dz;
        int64_t p;
#pragma omp parallel for schedule(static)
        for (p = 0; p < n; ++p) {
            if (lost && lost[p]) continue;
            int i, j, k;
            int64_t w[4], wl[2];
            if (!cic_weights(&g, x[p], y[p], &i, &j, w) ||
                !line_weights(sigma[p], nz, z_min, inv_dz, &k, wl)) {
                if (lost) lost[p] = 1;
                continue;
            }
            int64_t c00 = (int64_t)i * ny + j, c10 = c00 + ny, c01 = c00 + 1, c11 = c00 + ny + 1;
            int64_t s = ny + 2, f00 = (int64_t)(i + 1) * s + (j + 1);
            double exp_ = ((double)w[0] * ex[c00] + (double)w[1] * ex[c10] +
                           (double)w[2] * ex[c01] + (double)w[3] * ex[c11]) / ORC_CHARGE_ONE;
            double eyp = ((double)w[0] * ey[c00] + (double)w[1] * ey[c10] +
                          (double)w[2] * ey[c01] + (double)w[3] * ey[c11]) / ORC_CHARGE_ONE;
            double php = ((double)w[0] * phi[f00] + (double)w[1] * phi[f00 + s] +
                          (double)w[2] * phi[f00 + 1] + (double)w[3] * phi[f00 + s + 1]) /
                         ORC_CHARGE_ONE;
            double wp = ((double)wl[0] * lw[k] + (double)wl[1] * lw[k + 1]) / ORC_FRAC_ONE;
            double dp = ((double)wl[0] * ld[k] + (double)wl[1] * ld[k + 1]) / ORC_FRAC_ONE;
            px[p] += kappa * wp * exp_;
            py[p] += kappa * wp * eyp;
            psigma[p] -= gamma0 * kappa * php * dp;
        }
    }
    if (lw_out) memcpy(lw_out, lw, sizeof(double) * (size_t)nz);
    if (ld_out) memcpy(ld_out, ld, sizeof(double) * (size_t)nz);
    if (phi_out) memcpy(phi_out, phi, sizeof(double) * (size_t)(nx + 2) * (ny + 2));
done:
    free(q);
    free(h);
    free(phi);
    free(ex);
    free(ey);
    free(lw);
    free(ld);
    return n_in;
}

/* Tracking of a long bunch: as orc_track with the grounded pipe, every
 * space-charge element running orc_space_charge_line on the line of nz nodes
 * from z_min with spacing dz.  Returns -1 (nothing tracked) under the
 * conditions orc_push rejects, or when out of memory. */
int orc_track_line(int64_t n, double *x, double *px, double *y, double *py, double *sigma,
                   double *psigma, uint8_t *lost, int nx, int ny, double x_min, double y_min,
                   double dx, double dy, int nz, double z_min, double dz, double gamma0,
                   int n_el, const int32_t *kind, const double *par, int n_turns)
{
    double scale = 1.0 / (ORC_CHARGE_ONE * (double)n);
    if (!sigma || !psigma) return -1;
    for (int e = 0; e < n_el; ++e)
        if (kind[e] == ORC_SEXT_THICK && par[16 * e + 3] < 1.0) return -1;
    for (int t = 0; t < n_turns; ++t)
        for (int e = 0; e < n_el; ++e) {
            if (kind[e] == ORC_SC) {
                if (orc_space_charge_line(n, x, px, y, py, sigma, psigma, lost, nx, ny, x_min,
                                          y_min, dx, dy, nz, z_min, dz, gamma0, scale,
                                          par[16 * e], NULL, NULL, NULL) < 0)
                    return -1;
            } else {
                orc_push(n, x, px, y, py, sigma, psigma, lost, 1, kind + e, par + 16 * e);
            }
        }
    return 0;
}

/* Track n_turns through the element sequence of one turn: non-space-charge
 * elements are pushed, each space-charge element runs the full step above with
 * its own kappa.  The charge scale is 1/(2^24 n): n is the initial particle
 * count, so lost particles take their charge with them.  Returns -1 (nothing
 * tracked) under the conditions orc_push rejects. */
int orc_track_gather(int64_t n, double *x, double *px, double *y, double *py, double *sigma,
                     double *psigma, uint8_t *lost, const float *wt, int nx, int ny,
                     double x_min, double y_min, double dx, double dy, int n_el,
                     const int32_t *kind, const double *par, int n_turns, int pipe, int bspline);

int orc_track(int64_t n, double *x, double *px, double *y, double *py, double *sigma,
              double *psigma, uint8_t *lost, const float *wt, int nx, int ny, double x_min,
              double y_min, double dx, double dy, int n_el, const int32_t *kind,
              const double *par, int n_turns, int pipe)
{
    return orc_track_gather(n, x, px, y, py, sigma, psigma, lost, wt, nx, ny, x_min, y_min, dx,
                            dy, n_el, kind, par, n_turns, pipe, 0);
}

/* As orc_track; bspline != 0 takes every kick's field from the B-spline
 * surface of the potential (Sec. IV-C). */
int orc_track_gather(int64_t n, double *x, double *px, double *y, double *py, double *sigma,
                     double *psigma, uint8_t *lost, const float *wt, int nx, int ny,
                     double x_min, double y_min, double dx, double dy, int n_el,
                     const int32_t *kind, const double *par, int n_turns, int pipe, int bspline)
{
    double scale = 1.0 / (ORC_CHARGE_ONE * (double)n);
    for (int e = 0; e < n_el; ++e) {
        if (is_thick(kind[e]) && (!sigma || !psigma)) return -1;
        if (kind[e] == ORC_SEXT_THICK && par[16 * e + 3] < 1.0) return -1;
    }
    for (int t = 0; t < n_turns; ++t)
        for (int e = 0; e < n_el; ++e) {
            if (kind[e] == ORC_SC)
                space_charge_step(n, x, px, y, py, lost, wt, nx, ny, x_min, y_min, dx, dy, scale,
                                  par[16 * e], NULL, NULL, pipe, bspline);
            else
                orc_push(n, x, px, y, py, sigma, psigma, lost, 1, kind + e, par + 16 * e);
        }
    return 0;
}
