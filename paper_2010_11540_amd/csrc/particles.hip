// Particle-side kernels of libscpic for gfx950: the fused particle pass
// (gather + kick, push, cloud-in-cell deposit into an LDS tile of the charge
// grid) in its four- and six-dimensional forms, with the long-bunch line
// density or the B-spline field, single-beam and batched; and the copy
// between split and interleaved field layouts.
//
// Compiled with -ffp-contract=off: every FP64 expression below is evaluated
// as written, each operation correctly rounded, so the cell index, the
// fixed-point weights and a linear push are bit-identical to the same IEEE
// sums evaluated anywhere else.  The thick elements, which have no
// bit-identical counterpart, use explicit fused multiply-adds.
#include <algorithm>
#include <climits>
#include <vector>

#include "scpic_internal.h"

#pragma clang fp contract(off)

namespace scpic {
namespace {

constexpr int kWave = 64;

// Cell (i, j) holding the particle and its four fixed-point weights for the
// nodes (i,j), (i+1,j), (i,j+1), (i+1,j+1): the bilinear fractions of
// Sec. IV-A rounded to 12 bits per axis, summing to exactly 2^24.  False when
// the particle is outside [0, nx-1) x [0, ny-1) in node units (or NaN).
struct Cic {
    int i, j;
    uint32_t w00, w10, w01, w11;
};

__device__ __forceinline__ bool cic(const GridGeom &g, double x, double y, Cic &c)
{
    const double tx = (x - g.x_min) * g.inv_dx;
    const double ty = (y - g.y_min) * g.inv_dy;
    const bool in = tx >= 0.0 && tx < (double)(g.nx - 1) && ty >= 0.0 && ty < (double)(g.ny - 1);
    // outside (or NaN): evaluate on node 0 so the arithmetic below stays defined
    const double sx = in ? tx : 0.0, sy = in ? ty : 0.0;
    const double fi = floor(sx), fj = floor(sy);
    const uint32_t a = (uint32_t)(int)floor((sx - fi) * 4096.0 + 0.5);
    const uint32_t b = (uint32_t)(int)floor((sy - fj) * 4096.0 + 0.5);
    c.i = (int)fi;
    c.j = (int)fj;
    const uint32_t a0 = kFracOne - a, b0 = kFracOne - b;
    c.w00 = a0 * b0;
    c.w10 = a * b0;
    c.w01 = a0 * b;
    c.w11 = a * b;
    return in;
}

template <typename TE>
struct Vec2;
template <>
struct Vec2<double> {
    using type = double2;
};
template <>
struct Vec2<float> {
    using type = float2;
};

// Interpolated field at the particle from four (Ex, Ey) nodes: weights / 2^24
// applied in node order (i,j), (i+1,j), (i,j+1), (i+1,j+1).  row is the
// distance between rows i and i+1 in the node array.
template <typename V, typename TE>
__device__ __forceinline__ void gather_nodes(const V *e, int l00, int row, const Cic &c, TE &fx,
                                             TE &fy)
{
    const V e00 = e[l00], e10 = e[l00 + row], e01 = e[l00 + 1], e11 = e[l00 + row + 1];
    const TE w00 = (TE)c.w00, w10 = (TE)c.w10, w01 = (TE)c.w01, w11 = (TE)c.w11;
    fx = (w00 * e00.x + w10 * e10.x + w01 * e01.x + w11 * e11.x) * (TE)(1.0 / kChargeOne);
    fy = (w00 * e00.y + w10 * e10.y + w01 * e01.y + w11 * e11.y) * (TE)(1.0 / kChargeOne);
}

// Potential at the particle from its four nodes, as gather_nodes.
template <typename TE>
__device__ __forceinline__ TE gather_scalar(const TE *u, int l00, int row, const Cic &c)
{
    const TE w00 = (TE)c.w00, w10 = (TE)c.w10, w01 = (TE)c.w01, w11 = (TE)c.w11;
    return (w00 * u[l00] + w10 * u[l00 + row] + w01 * u[l00 + 1] + w11 * u[l00 + row + 1]) *
           (TE)(1.0 / kChargeOne);
}

// Field at (x, y) in cell c (c.i, c.j from cic()) from the bicubic B-spline
// surface of the node potential u (nodes -1..nx by -1..ny, row length ny + 2):
//   phi = sum_{m,n} u[i+m-1][j+n-1] B_m(tx) B_n(ty),  E = -grad phi,
// with the uniform cubic basis B_m on the exact cell fractions (not the
// 12-bit ones of the deposit); rows are contracted first.
template <typename TE>
__device__ __forceinline__ void bspline_field(const GridGeom &g, const TE *__restrict__ u,
                                              double x, double y, const Cic &c, TE &fx, TE &fy)
{
    const TE tx = (TE)((x - g.x_min) * g.inv_dx - (double)c.i);
    const TE ty = (TE)((y - g.y_min) * g.inv_dy - (double)c.j);
    TE bx[4], dbx[4], by[4], dby[4];
    auto basis = [](TE t, TE *b, TE *db) {
        const TE v = TE(1) - t, t2 = t * t;
        b[0] = v * v * v * TE(1.0 / 6.0);
        b[1] = (TE(3) * t2 * t - TE(6) * t2 + TE(4)) * TE(1.0 / 6.0);
        b[2] = (TE(-3) * t2 * t + TE(3) * t2 + TE(3) * t + TE(1)) * TE(1.0 / 6.0);
        b[3] = t2 * t * TE(1.0 / 6.0);
        db[0] = -v * v * TE(0.5);
        db[1] = (TE(3) * t2 - TE(4) * t) * TE(0.5);
        db[2] = (TE(-3) * t2 + TE(2) * t + TE(1)) * TE(0.5);
        db[3] = t2 * TE(0.5);
    };
    basis(tx, bx, dbx);
    basis(ty, by, dby);
    const int row = g.ny + 2;
    const TE *base = u + (size_t)c.i * row + c.j;  // node (i-1, j-1)
    TE v[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) v[m][n] = base[m * row + n];
    TE sx = 0, sy = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const TE r = v[m][0] * by[0] + v[m][1] * by[1] + v[m][2] * by[2] + v[m][3] * by[3];
        const TE d = v[m][0] * dby[0] + v[m][1] * dby[1] + v[m][2] * dby[2] + v[m][3] * dby[3];
        sx = sx + dbx[m] * r;
        sy = sy + bx[m] * d;
    }
    fx = -sx * (TE)g.inv_dx;
    fy = -sy * (TE)g.inv_dy;
}

// Node k of the line and the particle's two fixed-point line weights
// (4096 - a at k, a at k + 1): t = (sigma - z_min)(1/dz), k = floor(t),
// a = floor((t - k) 4096 + 0.5), the one-dimensional form of cic().  False
// outside [0, nz - 1) in node units (or NaN).
struct LineCic {
    int k;
    uint32_t w0, w1;
};

__device__ __forceinline__ bool line_cic(const LineSpec &L, double sg, LineCic &c)
{
    const double t = (sg - L.z_min) * L.inv_dz;
    const bool in = t >= 0.0 && t < (double)(L.nz - 1);
    const double st = in ? t : 0.0;
    const double fk = floor(st);
    const uint32_t a = (uint32_t)(int)floor((st - fk) * 4096.0 + 0.5);
    c.k = (int)fk;
    c.w0 = kFracOne - a;
    c.w1 = a;
    return in;
}

// One element applied to one particle (Sec. III): v <- M v for the linear
// maps, evaluated row by row left to right; the thin sextupole is the kick
// step of the split thick-sextupole integrator (Sec. III-C).
__device__ __forceinline__ void apply_element(int kind, const double *__restrict__ m, double &x,
                                              double &px, double &y, double &py)
{
    const double X = x, PX = px, Y = y, PY = py;
    if (kind == SCPIC_EL_LIN2X2) {
        x = m[0] * X + m[1] * PX;
        px = m[2] * X + m[3] * PX;
        y = m[4] * Y + m[5] * PY;
        py = m[6] * Y + m[7] * PY;
    } else if (kind == SCPIC_EL_LIN4X4) {
        x = m[0] * X + m[1] * PX + m[2] * Y + m[3] * PY;
        px = m[4] * X + m[5] * PX + m[6] * Y + m[7] * PY;
        y = m[8] * X + m[9] * PX + m[10] * Y + m[11] * PY;
        py = m[12] * X + m[13] * PX + m[14] * Y + m[15] * PY;
    } else if (kind == SCPIC_EL_SEXT_THIN) {
        const double k2l = m[0];
        px = PX - 0.5 * k2l * (X * X - Y * Y);
        py = PY + k2l * X * Y;
    }
}

// The thick elements below carry no bit-exactness contract (their reference
// evaluates other, equivalent formulas), so they use fused multiply-adds.

// sin and cos (HYP false) or sinh and cosh (HYP true) of phi0 + d from their
// values s0, c0 at phi0 and the Taylor series of the functions of d through
// d^11 and d^10 in Horner form (for |d| <= 1/16 the omitted terms are below
// 1e-19 of the result).
template <bool HYP>
__device__ __forceinline__ void shift_angle(double d, double s0, double c0, double &s, double &c)
{
    const double t = HYP ? d * d : -(d * d);
    double ps = fma(t, 1.0 / 39916800.0, 1.0 / 362880.0);
    ps = fma(t, ps, 1.0 / 5040.0);
    ps = fma(t, ps, 1.0 / 120.0);
    ps = fma(t, ps, 1.0 / 6.0);
    double pc = fma(t, 1.0 / 3628800.0, 1.0 / 40320.0);
    pc = fma(t, pc, 1.0 / 720.0);
    pc = fma(t, pc, 1.0 / 24.0);
    pc = fma(t, pc, 0.5);
    const double sd = fma(d * t, ps, d);
    const double cd = fma(t, pc, 1.0);
    s = fma(s0, cd, c0 * sd);
    c = HYP ? fma(c0, cd, s0 * sd) : fma(c0, cd, -(s0 * sd));
}

// One transverse plane of the thick quadrupole (Sec. III-B): u' = q p_u and
// p_u' = -K u with q = 1 - p_sigma (K = k1 for x, -k1 for y).  With C the
// plane's cos or cosh of its angle and sw = (sin or sinh)/sqrt(|K| q), the flow
// over L is u <- u C + q p_u sw, p_u <- p_u C - K u sw.  Returns the integral of
// p_u^2 over the element from the plane's invariant E = q p_u^2 + K u^2: since
// d(u p_u)/ds = 2 q p_u^2 - E, it is (E L + u(L) p_u(L) - u(0) p_u(0)) / (2 q);
// half_q = 1 / (2 q).
__device__ __forceinline__ double quad_plane(double &u, double &pu, double K, double q, double L,
                                             double C, double sw, double half_q)
{
    const double u0 = u, p0 = pu;
    u = fma(u0, C, q * p0 * sw);
    pu = fma(p0, C, -(K * u0 * sw));
    const double inv = fma(q * p0, p0, K * u0 * u0);
    return fma(inv, L, fma(u, pu, -(u0 * p0))) * half_q;
}

// Per-particle quantities every thick element of a pass shares: q = 1 - p_sigma,
// sqrt(q) and 1/sqrt(q).
struct Chroma {
    double psg, q, sq, isq;
};

__device__ __forceinline__ Chroma chroma(double psg)
{
    Chroma k;
    k.psg = psg;
    k.q = 1.0 - psg;
    // 1/sqrt(q) from the hardware estimate and two Newton steps (each about
    // doubles the correct bits), then sqrt(q) = q / sqrt(q): within a unit or
    // two of the last place, in a third of the instructions of a correctly
    // rounded square root and division (the thick elements carry no
    // bit-exactness contract; q <= 0 gives NaN either way)
    double y = __builtin_amdgcn_rsq(k.q);
    const double hq = -0.5 * k.q;
    y = y * fma(hq * y, y, 1.5);
    y = y * fma(hq * y, y, 1.5);
    k.isq = y;
    k.sq = k.q * y;
    return k;
}

// Thick quadrupole with chromatic focusing (Sec. III-B).  Both planes turn by
// phi = sqrt(|k1| q) L = phi0 sqrt(q): trigonometric functions in the
// focusing plane, hyperbolic in the other.  The host supplies phi0 and the
// four functions at phi0 (m[3..7]) and 1/sqrt|k1| (m[8]); a particle's
// functions follow from the offset d = phi - phi0 = phi0 (sqrt(q) - 1) by the
// addition formulas, with the series of the functions of d for |d| <= 1/16
// (any momentum spread of a real beam) and beyond that the series of d / 2^h
// doubled h times (the relative error grows about as 2^h units of rounding:
// 2^-46 at |d| = 64).  Then
//   sigma += p_sigma L / gamma0^2 - (1/2) int (px^2 + py^2) ds.
__device__ __forceinline__ void quad_thick(const double *__restrict__ m, double &x, double &px,
                                           double &y, double &py, double &sg, const Chroma &k)
{
    const double k1 = m[0], L = m[1], ig2 = m[2];
    const double q = k.q;
    double ix, iy;
    if (k1 == 0.0) {
        ix = px * px * L;
        iy = py * py * L;
        x = fma(q * px, L, x);
        y = fma(q * py, L, y);
    } else {
        const double phi0 = m[3], d = phi0 * (k.sq - 1.0);
        double s, c, sh, ch;
        if (fabs(d) <= 0.0625) {
            shift_angle<false>(d, m[4], m[5], s, c);
            shift_angle<true>(d, m[6], m[7], sh, ch);
        } else {
            // halve d into the series' range, double the angle back up, then
            // add phi0 (bounded: an infinite d ends in NaN, not a hang)
            int h = 0;
            double dh = d;
            while (h < 40 && fabs(dh) > 0.0625) {
                dh *= 0.5;
                ++h;
            }
            shift_angle<false>(dh, 0.0, 1.0, s, c);
            shift_angle<true>(dh, 0.0, 1.0, sh, ch);
            for (int r = 0; r < h; ++r) {
                const double s2 = 2.0 * s * c, c2 = fma(2.0 * c, c, -1.0);
                const double sh2 = 2.0 * sh * ch, ch2 = fma(2.0 * ch, ch, -1.0);
                s = s2;
                c = c2;
                sh = sh2;
                ch = ch2;
            }
            const double s0 = m[4], c0 = m[5], sh0 = m[6], ch0 = m[7];
            const double ns = fma(s0, c, c0 * s), nc = fma(c0, c, -(s0 * s));
            const double nsh = fma(sh0, ch, ch0 * sh), nch = fma(ch0, ch, sh0 * sh);
            s = ns;
            c = nc;
            sh = nsh;
            ch = nch;
        }
        const double iw = m[8] * k.isq;  // 1 / sqrt(|k1| q)
        const double half_q = 0.5 * k.isq * k.isq;
        if (k1 > 0.0) {
            ix = quad_plane(x, px, k1, q, L, c, s * iw, half_q);
            iy = quad_plane(y, py, -k1, q, L, ch, sh * iw, half_q);
        } else {
            ix = quad_plane(x, px, k1, q, L, ch, sh * iw, half_q);
            iy = quad_plane(y, py, -k1, q, L, c, s * iw, half_q);
        }
    }
    sg = sg + fma(k.psg * ig2, L, -0.5 * (ix + iy));
}

// One element applied to one particle in six dimensions (Sec. III): the
// four-dimensional elements as above (sigma, p_sigma untouched), the thick
// quadrupole with chromatic focusing (Sec. III-B), whose path length is
//   sigma += p_sigma L / gamma0^2 - (1/2) int (px^2 + py^2) ds,
// and the thick sextupole (Sec. III-C) as n symmetric products of the exact
// flows of H0 = (px^2 + py^2)(1 - p_sigma)/2 + p_sigma^2/(2 gamma0^2) and of
// V = k2 (x^3 - 3 x y^2)/6 over the step h = L/n:
//   H0 (a h), V (h/2), H0 (c h), V (h/2), H0 (a h),  c = 1/sqrt 3, a = (1 - c)/2.
// k2 = 0 takes the drift in one step; m[4] and m[5] are drift lengths the
// host folded into the first and last H0 flow, m[6..9] the step lengths it
// derived (the same for every particle).  p_sigma is constant in every
// element.
__device__ __forceinline__ void apply_element6(int kind, const double *__restrict__ m, double &x,
                                               double &px, double &y, double &py, double &sg,
                                               const Chroma &k)
{
    if (kind == SCPIC_EL_QUAD_THICK) {
        quad_thick(m, x, px, y, py, sg, k);
    } else if (kind == SCPIC_EL_SEXT_THICK && m[0] == 0.0) {
        // no sextupole field: the split composes to the exact drift of H0
        // over the whole length m[1] + m[4] + m[5], which the host put in m[6]
        const double L = m[6];
        sg = fma(fma(-0.5 * px, px, fma(-0.5 * py, py, k.psg * m[2])), L, sg);
        x = fma(px * k.q, L, x);
        y = fma(py * k.q, L, y);
    } else if (kind == SCPIC_EL_SEXT_THICK) {
        // the step h = m[1] / n and the split's a h, c h, k2 h / 2, computed
        // by the host in m[6..9]
        const int n = (int)m[3];
        const double dsg = k.psg * m[2];
        const double ta = m[7], tc = m[8], tv = m[9];
        auto drift = [&](double t) {
            x = fma(px * k.q, t, x);
            y = fma(py * k.q, t, y);
            sg = fma(fma(-0.5 * px, px, fma(-0.5 * py, py, dsg)), t, sg);
        };
        auto kick = [&]() {
            const double X = x, Y = y;
            px = fma(-0.5 * tv, fma(X, X, -(Y * Y)), px);
            py = fma(tv * X, Y, py);
        };
        // folded drifts (host side) lengthen the first and the last H0 flow
        const double lead = m[4], tail = m[5];
        for (int i = 0; i < n; ++i) {
            drift(i == 0 ? ta + lead : ta);
            kick();
            drift(tc);
            kick();
            drift(i == n - 1 ? ta + tail : ta);
        }
    } else {
        apply_element(kind, m, x, px, y, py);
    }
}

// Reductions over the 64 lanes of a wave with DPP row operations (no LDS
// traffic): the two quad permutations and the half-row and row mirrors leave
// every lane of a row of 16 holding its row's result; row broadcast 15 folds
// row 0 into row 1 and row 2 into row 3, row broadcast 31 folds row 1 into
// rows 2 and 3, so lane 63 holds the wave's result.  Rows a step does not
// write keep their value (the identity of the step's operation).
template <typename Op>
__device__ __forceinline__ int wave_reduce(int v, int identity, Op op)
{
    v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
    v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
    v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x141, 0xF, 0xF, false));  // row_half_mirror
    v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x140, 0xF, 0xF, false));  // row_mirror
    v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x142, 0xA, 0xF, false));  // row_bcast:15
    v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x143, 0xC, 0xF, false));  // row_bcast:31
    return __builtin_amdgcn_readlane(v, kWave - 1);
}
__device__ __forceinline__ int wave_min(int v)
{
    return wave_reduce(v, INT_MAX, [](int a, int b) { return min(a, b); });
}
__device__ __forceinline__ int wave_max(int v)
{
    return wave_reduce(v, INT_MIN, [](int a, int b) { return max(a, b); });
}
__device__ __forceinline__ int wave_sum(int v)
{
    return wave_reduce(v, 0, [](int a, int b) { return a + b; });
}

// t / w for 0 <= t < 2^16 and 1 <= w <= 2^16: the float product with the
// rounded reciprocal is within 0.01 of the quotient, so one integer step
// either way makes it exact.
__device__ __forceinline__ int div_small(int t, int w, float inv_w)
{
    int r = (int)((float)t * inv_w);
    r -= (r * w > t) ? 1 : 0;
    r += ((r + 1) * w <= t) ? 1 : 0;
    return r;
}

// A rectangle of grid nodes held in LDS: rows i0..i0+h-1, columns
// j0..j0+w-1, row-major with row length w.
struct Box {
    int i0, j0, h, w;
    // the four nodes of cell (i, j) lie inside
    __device__ __forceinline__ bool holds_cell(int i, int j) const
    {
        return i >= i0 && i + 1 < i0 + h && j >= j0 && j + 1 < j0 + w;
    }
    __device__ __forceinline__ int at(int i, int j) const { return (i - i0) * w + (j - j0); }
};

// Cells of the charge tile around a known box grown by `margin` cells and
// rounded to 4-column chunks, before any shrinking to a budget.
__device__ __forceinline__ int tile_cells(const GridGeom &g, const BlockHeader &h, int margin)
{
    const int i0 = max(0, h.i0 - margin), i1 = min(g.nx - 1, h.i1 + margin);
    const int j0 = max(0, h.j0 - margin) & ~3, j1 = min(g.ny - 1, h.j1 + margin) | 3;
    return (i1 - i0 + 1) * (j1 - j0 + 1);
}

constexpr int kTileMargin = 12;  // cells around the previous box (particles move)

// Charge tile of a workgroup: the bounding box of its previous deposit grown
// by `margin` cells (the particles move between steps), rounded to 4-column
// chunks, clamped to the grid and to the LDS budget; the whole grid when no
// previous box is known and the grid fits; else as much of the grid's centre
// as fits.  Cells outside the tile go to the global carry grid instead.
__device__ __forceinline__ Box charge_tile(const GridGeom &g, const BlockHeader &h, size_t budget,
                                           int margin)
{
    const int cap_cells = (int)min(budget / sizeof(uint32_t), (size_t)INT_MAX);
    Box t;
    const bool known = h.i0 >= 0 && h.i0 <= h.i1 && h.j0 >= 0 && h.j0 <= h.j1 && h.i1 < g.nx &&
                       h.j1 < g.ny;
    if (!known && g.nx * g.ny <= cap_cells) {
        t.i0 = 0;
        t.j0 = 0;
        t.h = g.nx;
        t.w = g.ny;
        return t;
    }
    int i0, i1, j0, j1;
    if (known) {
        i0 = max(0, h.i0 - margin);
        i1 = min(g.nx - 1, h.i1 + margin);
        j0 = max(0, h.j0 - margin);
        j1 = min(g.ny - 1, h.j1 + margin);
    } else {
        i0 = 0;
        i1 = g.nx - 1;
        j0 = 0;
        j1 = g.ny - 1;
    }
    j0 &= ~3;
    j1 |= 3;  // ny is a multiple of 4, so j1 stays inside the grid
    int w = j1 - j0 + 1, hgt = i1 - i0 + 1;
    // shrink symmetrically (rows first, then 4-column chunks) to the budget
    while (hgt * w > cap_cells && hgt > 2) {
        ++i0;
        if (hgt * w > cap_cells && hgt > 3) --i1;
        hgt = i1 - i0 + 1;
    }
    while (hgt * w > cap_cells && w > 8) {
        j0 += 4;
        w -= 4;
        if (hgt * w > cap_cells && w > 8) w -= 4;
    }
    t.i0 = i0;
    t.j0 = j0;
    t.h = hgt;
    t.w = w;
    return t;
}

// The fused particle pass.  Thread t of the launch (T threads in all) walks
// the particles p = t, t+T, t+2T, ...: consecutive lanes take consecutive
// particles, so every SoA load and store is coalesced, and the next
// particle's loads (the next two in the streamed form) are issued before the
// current one is worked on.  For each particle:
//   KICK     gather the node field at the particle with the deposit weights
//            and kick px, py by kappa * w_p * E (w_p = 1 without weights);
//            a particle found outside the domain is marked lost and frozen;
//   push     through els (uniform, read from the kernel arguments);
//   DEPOSIT  add the particle's four weights to the workgroup's LDS tile of
//            the charge grid (nodes outside the tile: global atomics on the
//            carry grid); particles outside the domain are marked lost.
// When the whole charge grid fits in LDS and the workgroup's threads have few
// particles each, the whole grid is the tile and gathers read the L2-resident
// field.  Otherwise the tile covers the box the workgroup's
// previous deposit recorded (its header; a workgroup owns the same particles
// at every step of a track), and that box of the field, which holds every
// node the kick gathers from, is staged in LDS beside the tile when it fits.
// At the end each workgroup writes the bounding box of its tile cells to its
// slice of the partials (no global atomics).
// MODE is a set of flags (0: four-dimensional).  1: the particles carry sigma
// and p_sigma and els may hold thick elements; sigma is loaded and stored with
// the transverse coordinates.  2: six-dimensional, with the long-bunch line
// density (Sec. IV): the kick is scaled by lambda/lambda_peak at the particle's sigma
// and p_sigma takes the longitudinal kick -gamma0 kappa phi lambda'/lambda_peak
// (both tables and the node potential phi from the last solve, interpolated
// with the particle's line and transverse weights); the deposit adds the
// particle's two line weights (the one-dimensional form of the charge
// assignment) to an LDS histogram flushed to the workgroup's row of
// line.partial.  A particle outside the line is lost like one outside the grid.
// 4: the kick's field is the analytic gradient of the bicubic B-spline surface
// of the node potential (Sec. IV-C), ef then pointing at the potential on
// nodes -1..nx by -1..ny.
// 8: the four transverse coordinates are streamed with non-temporal loads and
// stores (particle arrays far larger than the last-level cache, which they
// would only churn; smaller ones stay cached between passes).
// The body is shared by the single-beam kernel and the batched one: bid is
// the workgroup's index among the nblk workgroups working on beam P (its
// slice of the partials and its header), T = nblk * blockDim.x.
template <typename TE, bool KICK, bool DEPOSIT, int MODE>
__device__ __forceinline__ void pass_body(const ParticlePtrs &P, const GridGeom &g,
                                          const TE *__restrict__ ef, double kappa,
                                          const PassElements &els, const DepositTarget &dep,
                                          unsigned lds_bytes, int bid, int nblk,
                                          const LineSpec &line)
{
    using V = typename Vec2<TE>::type;
    constexpr bool LINE = (MODE & 2) != 0;
    constexpr bool SIX = (MODE & 1) != 0 || LINE;
    constexpr bool BSPL = (MODE & 4) != 0;
    constexpr bool NT = (MODE & 8) != 0;
    extern __shared__ __align__(16) unsigned char lds_all[];
    // LDS: [line histogram (MODE 2)][charge tile][staged field box].  The
    // histogram counts in 32 bits: a workgroup adds 4096 per particle and the
    // host launches no workgroup with more than 2^20 particles.
    const unsigned line_bytes = LINE ? ((unsigned)line.nz * 4u + 15u) & ~15u : 0u;
    uint32_t *lh = reinterpret_cast<uint32_t *>(lds_all);
    unsigned char *const lds = lds_all + line_bytes;
    lds_bytes -= line_bytes;
    __shared__ int s_box[4];
    __shared__ int s_count;
    // Six-dimensional passes read their elements' parameters from LDS (one
    // broadcast read per value) rather than from scalar registers, which the
    // thick elements' many parameters would otherwise spill.
    __shared__ double s_el[SIX ? kMaxPassElements * 16 : 1];
    static_assert(sizeof(s_el) + 256 <= kPassStaticLds, "static LDS beyond the reserved share");
    const int64_t T = (int64_t)nblk * blockDim.x;
    int64_t p = (int64_t)bid * blockDim.x + threadIdx.x;

    // first particle's loads go out before the LDS set-up
    double x = 0, px = 0, y = 0, py = 0, sg = 0, psg = 0;
    float wp = 1.0f;
    uint8_t lf = 1;
    if (p < P.n) {
        x = P.x[p];
        px = P.px[p];
        y = P.y[p];
        py = P.py[p];
        if constexpr (SIX) {
            sg = P.sigma[p];
            psg = P.psigma[p];
        }
        lf = P.lost ? P.lost[p] : 0;
        if (KICK && P.w) wp = P.w[p];
    }

    // When the whole charge grid fits in LDS and each thread has few
    // particles, the whole grid is the tile and the kick gathers from the
    // L2-resident field: the set-up then needs nothing from the previous pass
    // (no header read, no field staging), only the zeroing of the tile.
    // Otherwise the previous pass's header sizes the tile and the staged
    // field box, whose set-up pays off over many particles per thread.
    constexpr int64_t kWholeMaxPerThread = 4;
    const bool whole = DEPOSIT && (size_t)g.nx * g.ny <= lds_bytes / sizeof(uint32_t) &&
                       P.n <= kWholeMaxPerThread * T;
    BlockHeader hd;
    hd.i0 = -1;
    hd.i1 = -2;
    hd.j0 = -1;
    hd.j1 = -2;
    if ((KICK || DEPOSIT) && !whole) hd = dep.header[bid];
    // The kick stages the field over the previous box (every node it gathers
    // from) when that box fits in LDS beside the charge tile.
    const bool known = hd.i0 >= 0 && hd.i0 <= hd.i1 && hd.j0 >= 0 && hd.j0 <= hd.j1 &&
                       hd.i1 < g.nx && hd.j1 < g.ny;
    const Box fbox{hd.i0, hd.j0, hd.i1 - hd.i0 + 1, hd.j1 - hd.j0 + 1};
    const size_t field_bytes =
        (KICK && !BSPL && !whole && known) ? ((size_t)fbox.h * fbox.w + 2) * sizeof(V) : 0;
    // LDS layout: [charge tile][staged field box + 2 nodes of slack]
    Box tile{0, 0, 0, 0};
    size_t tile_bytes = 0;
    if constexpr (DEPOSIT) {
        // the widest margin (12, 8, 4 or 0 cells) that leaves room for the
        // field box; 12 when none does
        int margin = kTileMargin;
        if (field_bytes) {
            int m = kTileMargin;
            while (m >= 0 &&
                   sizeof(uint32_t) * (size_t)tile_cells(g, hd, m) + field_bytes > lds_bytes)
                m -= 4;
            if (m >= 0) margin = m;
        }
        tile = whole ? Box{0, 0, g.nx, g.ny} : charge_tile(g, hd, lds_bytes, margin);
        tile_bytes = sizeof(uint32_t) * (size_t)tile.h * tile.w;
    }
    uint32_t *lq = reinterpret_cast<uint32_t *>(lds);
    V *le = reinterpret_cast<V *>(lds + tile_bytes);
    Box ebox{0, 0, 0, 0};
    bool staged = false;
    if constexpr (KICK) {
        ebox = fbox;
        staged = field_bytes && field_bytes + tile_bytes <= (size_t)lds_bytes;
        if (field_bytes && !staged && tile_bytes < (size_t)lds_bytes) {
            // The whole box does not fit beside the tile: stage its centre,
            // as much as fits, when that keeps at least half of its nodes
            // (the box's edges hold only the tails of the distribution; a
            // particle outside the staged part gathers from L2).
            const int64_t room = (int64_t)(((size_t)lds_bytes - tile_bytes) / sizeof(V)) - 2;
            if (2 * room >= (int64_t)fbox.h * fbox.w) {
                int i0 = fbox.i0, i1 = fbox.i0 + fbox.h - 1, j0 = fbox.j0, j1 = fbox.j0 + fbox.w - 1;
                while ((int64_t)(i1 - i0 + 1) * (j1 - j0 + 1) > room) {
                    // trim the longer side, one node at each end
                    if (i1 - i0 >= j1 - j0) {
                        ++i0;
                        --i1;
                    } else {
                        ++j0;
                        --j1;
                    }
                }
                ebox = Box{i0, j0, i1 - i0 + 1, j1 - j0 + 1};
                staged = ebox.h >= 2 && ebox.w >= 2;
            }
        }
        if (staged) {
            // four nodes per thread per round; indices past the box repeat
            // its last node, so every load and store is unconditional and
            // the four loads are in flight before the first store
            const V *ev = reinterpret_cast<const V *>(ef);
            const int nodes = ebox.h * ebox.w;
            const int nt = (int)blockDim.x;
            const float inv_w = 1.0f / (float)ebox.w;
            auto node = [&](int t) {
                const int r = div_small(t, ebox.w, inv_w);
                return (ebox.i0 + r) * g.ny + ebox.j0 + (t - r * ebox.w);
            };
            for (int t0 = threadIdx.x; t0 < nodes; t0 += 4 * nt) {
                const int ta = t0, tb = min(t0 + nt, nodes - 1), tc = min(t0 + 2 * nt, nodes - 1),
                          td = min(t0 + 3 * nt, nodes - 1);
                const V va = ev[node(ta)], vb = ev[node(tb)], vc = ev[node(tc)], vd = ev[node(td)];
                le[ta] = va;
                le[tb] = vb;
                le[tc] = vc;
                le[td] = vd;
            }
        }
    }
    if constexpr (DEPOSIT) {
        const int n4 = tile.h * tile.w / 4;  // tile.w is a multiple of 4
        uint4 *q4 = reinterpret_cast<uint4 *>(lq);
        for (int t = threadIdx.x; t < n4; t += blockDim.x) q4[t] = make_uint4(0, 0, 0, 0);
        if constexpr (LINE)
            for (int t = threadIdx.x; t < line.nz; t += blockDim.x) lh[t] = 0u;
        if (threadIdx.x == 0) {
            s_box[0] = INT_MAX;
            s_box[1] = -1;
            s_box[2] = INT_MAX;
            s_box[3] = -1;
            s_count = 0;
        }
    }
    if constexpr (SIX)
        for (int t = threadIdx.x; t < els.n_el * 16; t += blockDim.x)
            s_el[t] = els.p[t >> 4][t & 15];
    if (KICK || DEPOSIT || SIX) __syncthreads();

    const bool moves = KICK || els.n_el > 0;
    int bi0 = INT_MAX, bi1 = -1, bj0 = INT_MAX, bj1 = -1, cnt = 0;
    // The streamed form keeps two particles in flight per lane ahead of the
    // one worked on (its loads come from memory, not the last-level cache):
    // the second is loaded here and moves up each iteration.
    static_assert(!NT || !SIX, "the streamed pass is four-dimensional");
    double xa = 0, pxa = 0, ya = 0, pya = 0;
    float wa = 1.0f;
    uint8_t lfa = 1;
    if constexpr (NT) {
        const int64_t pa = p + T;
        if (pa < P.n) {
            xa = __builtin_nontemporal_load(&P.x[pa]);
            pxa = __builtin_nontemporal_load(&P.px[pa]);
            ya = __builtin_nontemporal_load(&P.y[pa]);
            pya = __builtin_nontemporal_load(&P.py[pa]);
            lfa = P.lost ? P.lost[pa] : 0;
            if (KICK && P.w) wa = P.w[pa];
        }
    }
    for (; p < P.n; p += T) {
        const int64_t pn = p + (NT ? 2 : 1) * T;
        double xn = 0, pxn = 0, yn = 0, pyn = 0, sgn = 0, psgn = 0;
        float wn = 1.0f;
        uint8_t lfn = 1;
        if (pn < P.n) {
            if constexpr (NT) {
                xn = __builtin_nontemporal_load(&P.x[pn]);
                pxn = __builtin_nontemporal_load(&P.px[pn]);
                yn = __builtin_nontemporal_load(&P.y[pn]);
                pyn = __builtin_nontemporal_load(&P.py[pn]);
            } else {
                xn = P.x[pn];
                pxn = P.px[pn];
                yn = P.y[pn];
                pyn = P.py[pn];
            }
            if constexpr (SIX) {
                sgn = P.sigma[pn];
                psgn = P.psigma[pn];
            }
            lfn = P.lost ? P.lost[pn] : 0;
            if (KICK && P.w) wn = P.w[pn];
        }
        bool act = lf == 0;
        if (KICK && act) {
            Cic c;
            LineCic lc;
            const bool in = cic(g, x, y, c) && (!LINE || line_cic(line, sg, lc));
            if (in) {
                TE fx, fy;
                if constexpr (BSPL)
                    bspline_field(g, ef, x, y, c, fx, fy);
                else if (staged && ebox.holds_cell(c.i, c.j))
                    gather_nodes(le, ebox.at(c.i, c.j), ebox.w, c, fx, fy);
                else
                    gather_nodes(reinterpret_cast<const V *>(ef), c.i * g.ny + c.j, g.ny, c, fx, fy);
                if constexpr (LINE) {
                    const double w0 = (double)lc.w0, w1 = (double)lc.w1;
                    const double wl = (w0 * line.lw[lc.k] + w1 * line.lw[lc.k + 1]) / 4096.0;
                    const double dl = (w0 * line.ld[lc.k] + w1 * line.ld[lc.k + 1]) / 4096.0;
                    const TE fp = gather_scalar(reinterpret_cast<const TE *>(line.phi),
                                                (c.i + 1) * (g.ny + 2) + c.j + 1, g.ny + 2, c);
                    const double k = kappa * wl;
                    px = px + k * (double)fx;
                    py = py + k * (double)fy;
                    psg = psg - line.gamma0 * kappa * (double)fp * dl;
                } else {
                    const double k = kappa * (double)wp;
                    px = px + k * (double)fx;
                    py = py + k * (double)fy;
                }
            } else if (P.lost) {
                P.lost[p] = 1;
                act = false;
            }
        }
        if (act) {
            if constexpr (SIX) {
                const Chroma ck = chroma(psg);
                for (int e = 0; e < els.n_el; ++e)
                    apply_element6(els.kind[e], s_el + 16 * e, x, px, y, py, sg, ck);
            } else {
                for (int e = 0; e < els.n_el; ++e)
                    apply_element(els.kind[e], els.p[e], x, px, y, py);
            }
            if (moves) {
                // the kick changes only the momenta; the elements move the
                // particle (a kick-only pass writes px and py alone)
                const bool shifts = els.n_el > 0;
                if constexpr (NT) {
                    if (shifts) {
                        __builtin_nontemporal_store(x, &P.x[p]);
                        __builtin_nontemporal_store(y, &P.y[p]);
                    }
                    __builtin_nontemporal_store(px, &P.px[p]);
                    __builtin_nontemporal_store(py, &P.py[p]);
                } else {
                    if (shifts) {
                        P.x[p] = x;
                        P.y[p] = y;
                    }
                    P.px[p] = px;
                    P.py[p] = py;
                }
                if constexpr (SIX)
                    if (shifts) P.sigma[p] = sg;
                if constexpr (LINE && KICK) P.psigma[p] = psg;
            }
            if constexpr (DEPOSIT) {
                Cic c;
                LineCic lc;
                if (cic(g, x, y, c) && (!LINE || line_cic(line, sg, lc))) {
                    if constexpr (LINE) {
                        atomicAdd(&lh[lc.k], lc.w0);
                        atomicAdd(&lh[lc.k + 1], lc.w1);
                    }
                    if (tile.holds_cell(c.i, c.j)) {
                        // A 32-bit tile cell wraps after 2^32 units (256
                        // particles on one node); the atomic's old value
                        // shows the wrap and the lost 2^32 goes to the carry
                        // grid.  All four atomics issue before any check.
                        const int l = tile.at(c.i, c.j);
                        const int cg = c.i * g.ny + c.j;
                        const uint32_t o00 = atomicAdd(&lq[l], c.w00);
                        const uint32_t o10 = atomicAdd(&lq[l + tile.w], c.w10);
                        const uint32_t o01 = atomicAdd(&lq[l + 1], c.w01);
                        const uint32_t o11 = atomicAdd(&lq[l + tile.w + 1], c.w11);
                        if (o00 + c.w00 < o00) atomicAdd(&dep.carry[cg], 1ull << 32);
                        if (o10 + c.w10 < o10) atomicAdd(&dep.carry[cg + g.ny], 1ull << 32);
                        if (o01 + c.w01 < o01) atomicAdd(&dep.carry[cg + 1], 1ull << 32);
                        if (o11 + c.w11 < o11) atomicAdd(&dep.carry[cg + g.ny + 1], 1ull << 32);
                        bi0 = min(bi0, c.i);
                        bi1 = max(bi1, c.i + 1);
                        bj0 = min(bj0, c.j);
                        bj1 = max(bj1, c.j + 1);
                    } else {
                        const int cg = c.i * g.ny + c.j;
                        atomicAdd(&dep.carry[cg], (unsigned long long)c.w00);
                        atomicAdd(&dep.carry[cg + g.ny], (unsigned long long)c.w10);
                        atomicAdd(&dep.carry[cg + 1], (unsigned long long)c.w01);
                        atomicAdd(&dep.carry[cg + g.ny + 1], (unsigned long long)c.w11);
                    }
                    ++cnt;
                } else if (P.lost) {
                    P.lost[p] = 1;
                }
            }
        }
        if constexpr (NT) {
            x = xa;
            px = pxa;
            y = ya;
            py = pya;
            wp = wa;
            lf = lfa;
            xa = xn;
            pxa = pxn;
            ya = yn;
            pya = pyn;
            wa = wn;
            lfa = lfn;
        } else {
            x = xn;
            px = pxn;
            y = yn;
            py = pyn;
            if constexpr (SIX) {
                sg = sgn;
                psg = psgn;
            }
            wp = wn;
            lf = lfn;
        }
    }

    if constexpr (DEPOSIT) {
        // combine the lanes' boxes and counts, then copy the box of tile cells
        // to this workgroup's slice of the partials in 16-byte chunks (the
        // extra cells of the end chunks are zero and masked by the reader)
        bi0 = wave_min(bi0);
        bi1 = wave_max(bi1);
        bj0 = wave_min(bj0);
        bj1 = wave_max(bj1);
        cnt = wave_sum(cnt);
        if ((threadIdx.x & (kWave - 1)) == 0) {
            atomicMin(&s_box[0], bi0);
            atomicMax(&s_box[1], bi1);
            atomicMin(&s_box[2], bj0);
            atomicMax(&s_box[3], bj1);
            atomicAdd(&s_count, cnt);
        }
        __syncthreads();
        if constexpr (LINE)
            for (int t = threadIdx.x; t < line.nz; t += blockDim.x)
                line.partial[(size_t)bid * line.nz + t] = (unsigned long long)lh[t];
        const int i0 = s_box[0], i1 = s_box[1], j0 = s_box[2], j1 = s_box[3];
        if (i0 <= i1) {
            const int c0 = j0 >> 2, nch = (j1 >> 2) - c0 + 1;
            const int total = (i1 - i0 + 1) * nch;
            const float inv_nch = 1.0f / (float)nch;
            for (int t = threadIdx.x; t < total; t += blockDim.x) {
                const int r = div_small(t, nch, inv_nch);
                const int i = i0 + r, cc = c0 + (t - r * nch);
                const uint4 v = *reinterpret_cast<const uint4 *>(lq + tile.at(i, 4 * cc));
                reinterpret_cast<uint4 *>(dep.partial +
                                          ((size_t)i * dep.max_blocks + bid) * g.ny)[cc] = v;
            }
        }
        if (threadIdx.x == 0) {
            BlockHeader h;
            h.i0 = i0;
            h.i1 = i1;
            h.j0 = j0;
            h.j1 = j1;
            h.count = s_count;
            h.pad[0] = h.pad[1] = h.pad[2] = 0;
            dep.header[bid] = h;
        }
    }
}

// NT: the streamed form (four-dimensional passes only).
template <typename TE, bool KICK, bool DEPOSIT, bool SIX, bool NT = false>
__global__ void __launch_bounds__(1024)
    k_pass(ParticlePtrs P, GridGeom g, const TE *__restrict__ ef, double kappa,
           PassElements els, DepositTarget dep, unsigned lds_bytes)
{
    pass_body<TE, KICK, DEPOSIT, (SIX ? 1 : 0) | (NT ? 8 : 0)>(
        P, g, ef, kappa, els, dep, lds_bytes, (int)blockIdx.x, (int)gridDim.x, LineSpec{});
}

// The pass with the B-spline field (phi: the node potential on nodes -1..nx
// by -1..ny).
template <typename TE, bool KICK, bool DEPOSIT, bool SIX>
__global__ void __launch_bounds__(1024)
    k_pass_bspline(ParticlePtrs P, GridGeom g, const TE *__restrict__ phi, double kappa,
                   PassElements els, DepositTarget dep, unsigned lds_bytes)
{
    pass_body<TE, KICK, DEPOSIT, 4 | (SIX ? 1 : 0)>(P, g, phi, kappa, els, dep, lds_bytes,
                                                    (int)blockIdx.x, (int)gridDim.x, LineSpec{});
}

// The pass of a long bunch with its line density (six-dimensional).
template <typename TE, bool KICK, bool DEPOSIT>
__global__ void __launch_bounds__(1024)
    k_pass_line(ParticlePtrs P, GridGeom g, const TE *__restrict__ ef, double kappa,
                PassElements els, DepositTarget dep, unsigned lds_bytes, LineSpec line)
{
    pass_body<TE, KICK, DEPOSIT, 2>(P, g, ef, kappa, els, dep, lds_bytes, (int)blockIdx.x,
                                    (int)gridDim.x, line);
}

// One pass over every beam of a batch: workgroup -> beam from the batch's
// table, then the same body on that beam's particles, grid, field and
// partials with its own kick strength and elements (steps[beam]).
template <typename TE, bool KICK, bool DEPOSIT, bool SIX, bool NT = false>
__global__ void __launch_bounds__(1024)
    k_pass_batched(BatchLaunch b, ParticlePtrs all, const BatchStep *__restrict__ steps,
                   unsigned lds_bytes)
{
    const int k = b.pass_inst[blockIdx.x];
    const BatchInstance &I = b.inst[k];
    ParticlePtrs P;
    P.x = all.x + I.p0;
    P.px = all.px + I.p0;
    P.y = all.y + I.p0;
    P.py = all.py + I.p0;
    P.sigma = all.sigma ? all.sigma + I.p0 : nullptr;
    P.psigma = all.psigma ? all.psigma + I.p0 : nullptr;
    P.w = all.w ? all.w + I.p0 : nullptr;
    P.lost = all.lost ? all.lost + I.p0 : nullptr;
    P.n = I.n;
    P.stream = NT;
    pass_body<TE, KICK, DEPOSIT, (SIX ? 1 : 0) | (NT ? 8 : 0)>(
        P, I.g, (const TE *)I.ef, steps[k].kappa, steps[k].els, I.dep, lds_bytes,
        (int)blockIdx.x - I.pass_block0, I.pass_blocks, LineSpec{});
}

// Between two node arrays (ex, ey) and the internal interleaved layout ef
// (Ex, Ey per node), in either direction.
template <typename TE, bool TO_INTERLEAVED>
__global__ void __launch_bounds__(256)
    k_interleave(TE *__restrict__ ex, TE *__restrict__ ey, TE *__restrict__ ef, int ncell)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncell) {
        if (TO_INTERLEAVED) {
            ef[2 * c] = ex[c];
            ef[2 * c + 1] = ey[c];
        } else {
            ex[c] = ef[2 * c];
            ey[c] = ef[2 * c + 1];
        }
    }
}

// Dynamic LDS budgets of the four- and six-dimensional passes (the latter
// keep their element parameters in static LDS); set by prepare_pass_kernels.
size_t g_lds_limit = 0, g_lds_limit6 = 0;
template <bool SIX>
size_t lds_budget()
{
    return SIX ? g_lds_limit6 : g_lds_limit;
}

template <typename TE, bool KICK, bool DEPOSIT, bool SIX, bool NT = false>
hipError_t launch_pass_t(hipStream_t s, const ParticlePtrs &p, const GridGeom &g, const void *ef,
                         double kappa, const PassElements &els, const DepositTarget &dep,
                         int blocks, int threads)
{
    const size_t lds = (KICK || DEPOSIT) ? lds_budget<SIX>() : 0;
    hipLaunchKernelGGL((k_pass<TE, KICK, DEPOSIT, SIX, NT>), dim3(blocks), dim3(threads), lds, s,
                       p, g, (const TE *)ef, kappa, els, dep, (unsigned)lds);
    return hipGetLastError();
}

template <typename TE, bool KICK, bool DEPOSIT, bool SIX>
hipError_t launch_pass_bspline_t(hipStream_t s, const ParticlePtrs &p, const GridGeom &g,
                                 const void *phi, double kappa, const PassElements &els,
                                 const DepositTarget &dep, int blocks, int threads)
{
    const size_t lds = DEPOSIT ? lds_budget<SIX>() : 0;
    hipLaunchKernelGGL((k_pass_bspline<TE, KICK, DEPOSIT, SIX>), dim3(blocks), dim3(threads), lds,
                       s, p, g, (const TE *)phi, kappa, els, dep, (unsigned)lds);
    return hipGetLastError();
}

template <typename TE, bool KICK, bool DEPOSIT>
hipError_t launch_pass_line_t(hipStream_t s, const ParticlePtrs &p, const GridGeom &g,
                              const void *ef, double kappa, const PassElements &els,
                              const DepositTarget &dep, int blocks, int threads,
                              const LineSpec &line)
{
    hipLaunchKernelGGL((k_pass_line<TE, KICK, DEPOSIT>), dim3(blocks), dim3(threads), g_lds_limit6,
                       s, p, g, (const TE *)ef, kappa, els, dep, (unsigned)g_lds_limit6, line);
    return hipGetLastError();
}

template <typename TE, bool KICK, bool DEPOSIT, bool SIX, bool NT = false>
hipError_t launch_pass_batched_t(hipStream_t s, const BatchLaunch &b, const ParticlePtrs &all,
                                 const BatchStep *steps, int blocks, int threads)
{
    const size_t lds = (KICK || DEPOSIT) ? lds_budget<SIX>() : 0;
    hipLaunchKernelGGL((k_pass_batched<TE, KICK, DEPOSIT, SIX, NT>), dim3(blocks), dim3(threads),
                       lds, s, b, all, steps, (unsigned)lds);
    return hipGetLastError();
}

template <typename TE, bool SIX>
void pass_kernels_of(std::vector<const void *> &out)
{
    out.push_back((const void *)k_pass<TE, true, true, SIX>);
    out.push_back((const void *)k_pass<TE, false, true, SIX>);
    out.push_back((const void *)k_pass<TE, true, false, SIX>);
    out.push_back((const void *)k_pass_batched<TE, true, true, SIX>);
    out.push_back((const void *)k_pass_batched<TE, false, true, SIX>);
    out.push_back((const void *)k_pass_batched<TE, true, false, SIX>);
    out.push_back((const void *)k_pass_bspline<TE, true, true, SIX>);
    if (!SIX) {
        out.push_back((const void *)k_pass<TE, true, true, false, true>);
        out.push_back((const void *)k_pass<TE, false, true, false, true>);
        out.push_back((const void *)k_pass<TE, true, false, false, true>);
        out.push_back((const void *)k_pass_batched<TE, true, true, false, true>);
        out.push_back((const void *)k_pass_batched<TE, false, true, false, true>);
        out.push_back((const void *)k_pass_batched<TE, true, false, false, true>);
    }
    if (SIX) {
        out.push_back((const void *)k_pass_line<TE, true, true>);
        out.push_back((const void *)k_pass_line<TE, false, true>);
        out.push_back((const void *)k_pass_line<TE, true, false>);
    }
}

}  // namespace

bool has_thick(const PassElements &els)
{
    for (int e = 0; e < els.n_el; ++e)
        if (els.kind[e] == SCPIC_EL_QUAD_THICK || els.kind[e] == SCPIC_EL_SEXT_THICK) return true;
    return false;
}

// Allow the passes the dynamic LDS they use (beyond the default limit): the
// device's per-workgroup LDS (lds_per_workgroup) minus the kernels' static
// LDS, at most 256 bytes for the four-dimensional passes and kPassStaticLds
// for the six-dimensional ones.  Called once per context, outside any stream
// capture.
hipError_t prepare_pass_kernels(size_t lds_per_workgroup)
{
    g_lds_limit = lds_per_workgroup - 256;
    g_lds_limit6 = lds_per_workgroup - kPassStaticLds;
    std::vector<const void *> four, six;
    pass_kernels_of<double, false>(four);
    pass_kernels_of<float, false>(four);
    pass_kernels_of<double, true>(six);
    pass_kernels_of<float, true>(six);
    for (const void *k : four) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)g_lds_limit);
        if (e != hipSuccess) return e;
    }
    for (const void *k : six) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)g_lds_limit6);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The runtime flags as template arguments: L(TE, KICK, DEPOSIT, SIX) expands
// to the launch of the matching instantiation.
#define SCPIC_DISPATCH(L)                                                                     \
    if (mixed) {                                                                              \
        if (six)                                                                              \
            return kick ? (deposit ? L(float, true, true, true) : L(float, true, false, true)) \
                        : (deposit ? L(float, false, true, true)                              \
                                   : L(float, false, false, true));                           \
        return kick ? (deposit ? L(float, true, true, false) : L(float, true, false, false))  \
                    : (deposit ? L(float, false, true, false) : L(float, false, false, false)); \
    }                                                                                         \
    if (six)                                                                                  \
        return kick ? (deposit ? L(double, true, true, true) : L(double, true, false, true))  \
                    : (deposit ? L(double, false, true, true) : L(double, false, false, true)); \
    return kick ? (deposit ? L(double, true, true, false) : L(double, true, false, false))    \
                : (deposit ? L(double, false, true, false) : L(double, false, false, false))

// The four-dimensional kernels by precision, kick and deposit.
#define SCPIC_DISPATCH4(L)                                                                \
    if (mixed)                                                                            \
        return kick ? (deposit ? L(float, true, true) : L(float, true, false))            \
                    : (deposit ? L(float, false, true) : L(float, false, false));         \
    return kick ? (deposit ? L(double, true, true) : L(double, true, false))              \
                : (deposit ? L(double, false, true) : L(double, false, false))

hipError_t launch_pass(hipStream_t s, const ParticlePtrs &p, const GridGeom &g, bool kick,
                       bool mixed, const void *ef, double kappa, const PassElements &els,
                       bool deposit, const DepositTarget &dep, int blocks, int threads,
                       const LineSpec *line, const void *bspline_phi)
{
    if (blocks <= 0) return hipSuccess;
    if (bspline_phi && kick) {
        const bool six = has_thick(els);
#define SCPIC_LB(T, D, S) \
    launch_pass_bspline_t<T, true, D, S>(s, p, g, bspline_phi, kappa, els, dep, blocks, threads)
        if (mixed)
            return six ? (deposit ? SCPIC_LB(float, true, true) : SCPIC_LB(float, false, true))
                       : (deposit ? SCPIC_LB(float, true, false) : SCPIC_LB(float, false, false));
        return six ? (deposit ? SCPIC_LB(double, true, true) : SCPIC_LB(double, false, true))
                   : (deposit ? SCPIC_LB(double, true, false) : SCPIC_LB(double, false, false));
#undef SCPIC_LB
    }
    if (line && (kick || deposit)) {
#define SCPIC_LL(T)                                                                             \
    (kick ? (deposit ? launch_pass_line_t<T, true, true>(s, p, g, ef, kappa, els, dep, blocks,  \
                                                         threads, *line)                        \
                     : launch_pass_line_t<T, true, false>(s, p, g, ef, kappa, els, dep, blocks, \
                                                          threads, *line))                      \
          : launch_pass_line_t<T, false, true>(s, p, g, ef, kappa, els, dep, blocks, threads,   \
                                               *line))
        return mixed ? SCPIC_LL(float) : SCPIC_LL(double);
#undef SCPIC_LL
    }
    const bool six = has_thick(els);
    if (!six && p.stream) {
#define SCPIC_L(T, K, D) \
    launch_pass_t<T, K, D, false, true>(s, p, g, ef, kappa, els, dep, blocks, threads)
        SCPIC_DISPATCH4(SCPIC_L);
#undef SCPIC_L
    }
#define SCPIC_L(T, K, D, S) launch_pass_t<T, K, D, S>(s, p, g, ef, kappa, els, dep, blocks, threads)
    SCPIC_DISPATCH(SCPIC_L);
#undef SCPIC_L
}

hipError_t launch_pass_batched(hipStream_t s, const BatchLaunch &b, const ParticlePtrs &all,
                               const BatchStep *steps, bool kick, bool mixed, bool deposit,
                               bool six, int blocks, int threads)
{
    if (blocks <= 0) return hipSuccess;
    if (!six && all.stream) {
#define SCPIC_L(T, K, D) \
    launch_pass_batched_t<T, K, D, false, true>(s, b, all, steps, blocks, threads)
        SCPIC_DISPATCH4(SCPIC_L);
#undef SCPIC_L
    }
#define SCPIC_L(T, K, D, S) launch_pass_batched_t<T, K, D, S>(s, b, all, steps, blocks, threads)
    SCPIC_DISPATCH(SCPIC_L);
#undef SCPIC_L
}
#undef SCPIC_DISPATCH
#undef SCPIC_DISPATCH4

namespace {

constexpr int kMomentThreads = 256;

// One pass of the beam moments over the alive particles (diagnostics, not on
// the step's path).  PASS 1 sums 1, x, px, y, py; PASS 2 sums the products
// of the deviations from the means first[1..4] / first[0].  Each workgroup
// reduces its threads in a fixed tree and writes part[block][k].
template <int PASS>
__global__ void __launch_bounds__(kMomentThreads)
    k_moments(ParticlePtrs P, const double *__restrict__ first, double *__restrict__ part)
{
    double acc[kMoments] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double mx = 0.0, mpx = 0.0, my = 0.0, mpy = 0.0;
    if (PASS == 2 && first[0] > 0.0) {
        mx = first[1] / first[0];
        mpx = first[2] / first[0];
        my = first[3] / first[0];
        mpy = first[4] / first[0];
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P.n; p += stride) {
        if (P.lost && P.lost[p]) continue;
        const double x = P.x[p], px = P.px[p], y = P.y[p], py = P.py[p];
        if (PASS == 1) {
            acc[0] += 1.0;
            acc[1] += x;
            acc[2] += px;
            acc[3] += y;
            acc[4] += py;
        } else {
            const double dx = x - mx, dpx = px - mpx, dy = y - my, dpy = py - mpy;
            acc[0] += dx * dx;
            acc[1] += dpx * dpx;
            acc[2] += dx * dpx;
            acc[3] += dy * dy;
            acc[4] += dpy * dpy;
            acc[5] += dy * dpy;
        }
    }
    __shared__ double red[kMoments][kMomentThreads];
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < kMoments; ++k) red[k][t] = acc[k];
    __syncthreads();
    for (int h = kMomentThreads / 2; h > 0; h >>= 1) {
        if (t < h)
#pragma unroll
            for (int k = 0; k < kMoments; ++k) red[k][t] += red[k][t + h];
        __syncthreads();
    }
    if (t < kMoments) part[(size_t)blockIdx.x * kMoments + t] = red[t][0];
}

// The workgroups' sums added in block order.
__global__ void __launch_bounds__(64) k_moments_sum(const double *__restrict__ part, int nblocks,
                                                   double *__restrict__ out)
{
    const int k = threadIdx.x;
    if (k < kMoments) {
        double s = 0.0;
        for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * kMoments + k];
        out[k] = s;
    }
}

}  // namespace

hipError_t launch_moments(hipStream_t s, const ParticlePtrs &p, double *part, double *sums)
{
    hipLaunchKernelGGL(k_moments<1>, dim3(kMomentBlocks), dim3(kMomentThreads), 0, s, p,
                       (const double *)nullptr, part);
    hipLaunchKernelGGL(k_moments_sum, dim3(1), dim3(64), 0, s, (const double *)part,
                       kMomentBlocks, sums);
    hipLaunchKernelGGL(k_moments<2>, dim3(kMomentBlocks), dim3(kMomentThreads), 0, s, p,
                       (const double *)sums, part);
    hipLaunchKernelGGL(k_moments_sum, dim3(1), dim3(64), 0, s, (const double *)part,
                       kMomentBlocks, sums + kMoments);
    return hipGetLastError();
}

hipError_t launch_interleave(hipStream_t s, bool mixed, bool to_interleaved, void *ex, void *ey,
                             void *ef, int ncell)
{
    const dim3 grid((ncell + 255) / 256);
    if (mixed) {
        if (to_interleaved)
            hipLaunchKernelGGL((k_interleave<float, true>), grid, dim3(256), 0, s, (float *)ex,
                               (float *)ey, (float *)ef, ncell);
        else
            hipLaunchKernelGGL((k_interleave<float, false>), grid, dim3(256), 0, s, (float *)ex,
                               (float *)ey, (float *)ef, ncell);
    } else {
        if (to_interleaved)
            hipLaunchKernelGGL((k_interleave<double, true>), grid, dim3(256), 0, s, (double *)ex,
                               (double *)ey, (double *)ef, ncell);
        else
            hipLaunchKernelGGL((k_interleave<double, false>), grid, dim3(256), 0, s, (double *)ex,
                               (double *)ey, (double *)ef, ncell);
    }
    return hipGetLastError();
}

}  // namespace scpic
