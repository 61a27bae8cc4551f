// Particle-side kernels of libscpic for gfx950: the fused particle pass
// (gather + kick, push, cloud-in-cell deposit into LDS) and the reduction of
// the per-block charge partials.
//
// Compiled with -ffp-contract=off: every FP64 expression below is evaluated
// as written, each operation correctly rounded, so the cell index, the
// fixed-point weights and a linear push are bit-identical to the same IEEE
// sums evaluated anywhere else.
#include <algorithm>
#include <climits>

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
    if (!(tx >= 0.0 && tx < (double)(g.nx - 1))) return false;
    if (!(ty >= 0.0 && ty < (double)(g.ny - 1))) return false;
    const double fi = floor(tx), fj = floor(ty);
    const uint32_t a = (uint32_t)(int)floor((tx - fi) * 4096.0 + 0.5);
    const uint32_t b = (uint32_t)(int)floor((ty - fj) * 4096.0 + 0.5);
    c.i = (int)fi;
    c.j = (int)fj;
    const uint32_t a0 = kFracOne - a, b0 = kFracOne - b;
    c.w00 = a0 * b0;
    c.w10 = a * b0;
    c.w01 = a0 * b;
    c.w11 = a * b;
    return true;
}

// Interpolated field at the particle from the interleaved node field
// (e[2c] = Ex, e[2c+1] = Ey, one 2-vector load per node): weights / 2^24
// applied to the four nodes, summed in node order (i,j), (i+1,j), (i,j+1),
// (i+1,j+1).
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

template <typename TE>
__device__ __forceinline__ void gather(const TE *__restrict__ e, int c00, int ny, const Cic &c,
                                       TE &fx, TE &fy)
{
    using V = typename Vec2<TE>::type;
    const V *ev = reinterpret_cast<const V *>(e);
    const V e00 = ev[c00], e10 = ev[c00 + ny], e01 = ev[c00 + 1], e11 = ev[c00 + ny + 1];
    const TE w00 = (TE)c.w00, w10 = (TE)c.w10, w01 = (TE)c.w01, w11 = (TE)c.w11;
    fx = (w00 * e00.x + w10 * e10.x + w01 * e01.x + w11 * e11.x) * (TE)(1.0 / kChargeOne);
    fy = (w00 * e00.y + w10 * e10.y + w01 * e01.y + w11 * e11.y) * (TE)(1.0 / kChargeOne);
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

// Add a particle's four weights to the LDS charge grid.  A 32-bit cell wraps
// after 2^32 units (256 particles sitting exactly on one node); the returned
// old value shows a wrap, and the lost 2^32 goes to the global carry grid,
// which the reduction adds back.  All four atomics are issued before any
// return value is inspected.  Wraps need that many particles of one
// workgroup on one node, so the global atomic is rare.
__device__ __forceinline__ void lds_deposit(uint32_t *q, int c00, int ny, const Cic &c,
                                            unsigned long long *__restrict__ carry)
{
    const uint32_t o00 = atomicAdd(&q[c00], c.w00);
    const uint32_t o10 = atomicAdd(&q[c00 + ny], c.w10);
    const uint32_t o01 = atomicAdd(&q[c00 + 1], c.w01);
    const uint32_t o11 = atomicAdd(&q[c00 + ny + 1], c.w11);
    if (o00 + c.w00 < o00) atomicAdd(&carry[c00], 1ull << 32);
    if (o10 + c.w10 < o10) atomicAdd(&carry[c00 + ny], 1ull << 32);
    if (o01 + c.w01 < o01) atomicAdd(&carry[c00 + 1], 1ull << 32);
    if (o11 + c.w11 < o11) atomicAdd(&carry[c00 + ny + 1], 1ull << 32);
}

__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, kWave));
    return v;
}
__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
    return v;
}
__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Combine the lanes' bounding boxes and counts, then write the workgroup's
// box of LDS cells to its slice of the partials and its header.
__device__ __forceinline__ void flush_partials(const GridGeom &g, const DepositTarget &dep,
                                               const uint32_t *lds_q, int *s_box, int *s_count,
                                               int bi0, int bi1, int bj0, int bj1, int cnt)
{
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
        atomicAdd(s_count, cnt);
    }
    __syncthreads();
    const int i0 = s_box[0], i1 = s_box[1], j0 = s_box[2], j1 = s_box[3];
    if (i0 <= i1) {
        // whole 16-byte chunks (4 cells) covering columns j0..j1 of each row;
        // the extra cells of the end chunks are zero here and masked by the
        // reader
        const int c0 = j0 >> 2, nch = (j1 >> 2) - c0 + 1;
        const int total = (i1 - i0 + 1) * nch;
        for (int t = threadIdx.x; t < total; t += blockDim.x) {
            const int r = t / nch;
            const int i = i0 + r, cc = c0 + (t - r * nch);
            const uint4 v = reinterpret_cast<const uint4 *>(lds_q + (size_t)i * g.ny)[cc];
            reinterpret_cast<uint4 *>(dep.partial +
                                      ((size_t)i * dep.max_blocks + blockIdx.x) * g.ny)[cc] = v;
        }
    }
    if (threadIdx.x == 0) {
        BlockHeader h;
        h.i0 = i0;
        h.i1 = i1;
        h.j0 = j0;
        h.j1 = j1;
        h.count = *s_count;
        h.pad[0] = h.pad[1] = h.pad[2] = 0;
        dep.header[blockIdx.x] = h;
    }
}

// Gather from a field box staged in LDS (row width w), same order and
// arithmetic as gather().
template <typename V, typename TE>
__device__ __forceinline__ void gather_lds(const V *le, int l00, int w, const Cic &c, TE &fx,
                                           TE &fy)
{
    const V e00 = le[l00], e10 = le[l00 + w], e01 = le[l00 + 1], e11 = le[l00 + w + 1];
    const TE w00 = (TE)c.w00, w10 = (TE)c.w10, w01 = (TE)c.w01, w11 = (TE)c.w11;
    fx = (w00 * e00.x + w10 * e10.x + w01 * e01.x + w11 * e11.x) * (TE)(1.0 / kChargeOne);
    fy = (w00 * e00.y + w10 * e10.y + w01 * e01.y + w11 * e11.y) * (TE)(1.0 / kChargeOne);
}

// The fused particle pass.  Thread t of the launch (T threads in all) takes
// the particles t + u*T + k*U*T, u < U: consecutive lanes take consecutive
// particles, so every SoA load and store is coalesced, and each thread issues
// the loads of its U particles before using any.  For each particle:
//   KICK     gather the node field at the particle with the deposit weights
//            and kick px, py by kappa * E (a particle found outside the domain
//            is marked lost and frozen);
//   push     through els (uniform, read from the kernel arguments);
//   DEPOSIT  add the particle's four weights to the workgroup's private copy
//            of the charge grid in LDS (particles outside are marked lost).
// At the end each workgroup writes the bounding box of the cells it touched
// to its own slice of the partials (no global atomics).
//
// When the launch covers every particle in one batch (n <= U*T), a workgroup
// owns the same particles at every step, so the bounding box its previous
// deposit recorded holds every node its kick gathers from: that box of the
// field is staged in LDS with coalesced loads, and the random gathers hit LDS
// instead of the L1/L2 path.  A particle outside the staged box (a stale or
// oversized box) takes the global gather, so the box only affects speed.  The
// LDS of the staged field is reused for the charge grid once the kicks are
// done; coordinates are stored right after the push, before the deposit.
template <typename TE>
struct NodeStage {
    int i0, j0, w, h;  // staged rows i0..i0+h-1, columns j0..j0+w-1
    bool on;
};

template <typename TE, bool KICK, bool DEPOSIT, int U>
__device__ __forceinline__ void pass_single_batch(const ParticlePtrs &P, const GridGeom &g,
                                                  const TE *__restrict__ ef, double kappa,
                                                  const PassElements &els, const DepositTarget &dep,
                                                  unsigned char *lds, size_t lds_bytes, int *s_box,
                                                  int *s_count)
{
    using V = typename Vec2<TE>::type;
    const int ncell = g.nx * g.ny;
    const int64_t T = (int64_t)gridDim.x * blockDim.x;
    const int64_t base = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double x[U], px[U], y[U], py[U];
    bool act[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t p = base + u * T;
        act[u] = p < P.n;
        uint8_t lf = 0;
        if (act[u]) {
            x[u] = P.x[p];
            px[u] = P.px[p];
            y[u] = P.y[p];
            py[u] = P.py[p];
            if (P.lost) lf = P.lost[p];
        }
        act[u] = act[u] && lf == 0;
    }
    // LDS: the charge grid first, then (when it fits beside it) the staged
    // field box; a box that only fits alone shares the grid's space and the
    // grid is zeroed after the kicks.
    uint32_t *lds_q = reinterpret_cast<uint32_t *>(lds);
    const size_t qbytes = DEPOSIT ? sizeof(uint32_t) * (size_t)ncell : 0;
    NodeStage<TE> st;
    st.on = false;
    bool aliased = false;
    const V *le = nullptr;
    if constexpr (KICK) {
        const BlockHeader h = dep.header[blockIdx.x];
        st.i0 = h.i0;
        st.j0 = h.j0;
        st.h = h.i1 - h.i0 + 1;
        st.w = h.j1 - h.j0 + 1;
        const bool valid = h.i0 >= 0 && h.j0 >= 0 && h.i1 < g.nx && h.j1 < g.ny && st.h > 0 &&
                           st.w > 0;
        const size_t need = valid ? (size_t)st.h * st.w * sizeof(V) : 0;
        V *dst = nullptr;
        if (valid && need <= lds_bytes - qbytes) {
            st.on = true;
            dst = reinterpret_cast<V *>(lds + qbytes);
        } else if (valid && need <= lds_bytes) {
            st.on = true;
            aliased = DEPOSIT;
            dst = reinterpret_cast<V *>(lds);
        }
        if (st.on) {
            // four nodes per thread per round, all loads before the stores
            const V *ev = reinterpret_cast<const V *>(ef);
            const int nodes = st.h * st.w;
            const int nt = (int)blockDim.x;
            for (int t0 = threadIdx.x; t0 < nodes; t0 += 4 * nt) {
                V v[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int t = t0 + k * nt;
                    const int r = t / st.w;
                    v[k] = t < nodes ? ev[(st.i0 + r) * g.ny + st.j0 + (t - r * st.w)] : V{};
                }
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (t0 + k * nt < nodes) dst[t0 + k * nt] = v[k];
            }
        }
        le = dst;
    }
    if (DEPOSIT && !aliased) {
        uint4 *q4 = reinterpret_cast<uint4 *>(lds_q);
        for (int t = threadIdx.x; t < ncell / 4; t += blockDim.x) q4[t] = make_uint4(0, 0, 0, 0);
        if (threadIdx.x == 0) {
            s_box[0] = INT_MAX;
            s_box[1] = -1;
            s_box[2] = INT_MAX;
            s_box[3] = -1;
            *s_count = 0;
        }
    }
    __syncthreads();  // staged field and zeroed charge grid ready
    if constexpr (KICK) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!act[u]) continue;
            Cic c;
            if (cic(g, x[u], y[u], c)) {
                TE fx, fy;
                const int li = c.i - st.i0, lj = c.j - st.j0;
                if (st.on && li >= 0 && li + 1 < st.h && lj >= 0 && lj + 1 < st.w)
                    gather_lds(le, li * st.w + lj, st.w, c, fx, fy);
                else
                    gather(ef, c.i * g.ny + c.j, g.ny, c, fx, fy);
                px[u] = px[u] + kappa * (double)fx;
                py[u] = py[u] + kappa * (double)fy;
            } else if (P.lost) {
                P.lost[base + u * T] = 1;
                act[u] = false;
            }
        }
    }
    for (int e = 0; e < els.n_el; ++e) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (act[u]) apply_element(els.kind[e], els.p[e], x[u], px[u], y[u], py[u]);
    }
    if (KICK || els.n_el > 0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!act[u]) continue;
            const int64_t p = base + u * T;
            P.x[p] = x[u];
            P.px[p] = px[u];
            P.y[p] = y[u];
            P.py[p] = py[u];
        }
    }
    if constexpr (DEPOSIT) {
        if (aliased) {
            __syncthreads();  // every kick has read the staged field
            uint4 *q4 = reinterpret_cast<uint4 *>(lds_q);
            for (int t = threadIdx.x; t < ncell / 4; t += blockDim.x)
                q4[t] = make_uint4(0, 0, 0, 0);
            if (threadIdx.x == 0) {
                s_box[0] = INT_MAX;
                s_box[1] = -1;
                s_box[2] = INT_MAX;
                s_box[3] = -1;
                *s_count = 0;
            }
            __syncthreads();
        }
        int bi0 = INT_MAX, bi1 = -1, bj0 = INT_MAX, bj1 = -1, cnt = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!act[u]) continue;
            Cic c;
            if (cic(g, x[u], y[u], c)) {
                lds_deposit(lds_q, c.i * g.ny + c.j, g.ny, c, dep.carry);
                bi0 = min(bi0, c.i);
                bi1 = max(bi1, c.i + 1);
                bj0 = min(bj0, c.j);
                bj1 = max(bj1, c.j + 1);
                ++cnt;
            } else if (P.lost) {
                P.lost[base + u * T] = 1;
            }
        }
        flush_partials(g, dep, lds_q, s_box, s_count, bi0, bi1, bj0, bj1, cnt);
    }
}

// Streaming path: each thread walks its particles p = t, t+T, ... one at a
// time, issuing the loads of the next particle before working on the
// current one, so loads, LDS work and stores of different particles overlap.
// The staged field box (when it fits beside the charge grid) and the zeroed
// grid are prepared once, before the walk.
template <typename TE, bool KICK, bool DEPOSIT>
__device__ __forceinline__ void pass_stream(const ParticlePtrs &P, const GridGeom &g,
                                            const TE *__restrict__ ef, double kappa,
                                            const PassElements &els, const DepositTarget &dep,
                                            unsigned char *lds, size_t lds_bytes, int *s_box,
                                            int *s_count)
{
    using V = typename Vec2<TE>::type;
    const int ncell = g.nx * g.ny;
    const int64_t T = (int64_t)gridDim.x * blockDim.x;
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // first particle's loads go out before the LDS preparation
    double x = 0, px = 0, y = 0, py = 0;
    uint8_t lf = 1;
    if (p < P.n) {
        x = P.x[p];
        px = P.px[p];
        y = P.y[p];
        py = P.py[p];
        lf = P.lost ? P.lost[p] : 0;
    }
    uint32_t *lds_q = reinterpret_cast<uint32_t *>(lds);
    const size_t qbytes = DEPOSIT ? sizeof(uint32_t) * (size_t)ncell : 0;
    NodeStage<TE> st;
    st.on = false;
    st.i0 = st.j0 = 0;
    st.h = st.w = 0;
    const V *le = nullptr;
    if constexpr (KICK) {
        const BlockHeader h = dep.header[blockIdx.x];
        const int hh = h.i1 - h.i0 + 1, ww = h.j1 - h.j0 + 1;
        const bool valid = h.i0 >= 0 && h.j0 >= 0 && h.i1 < g.nx && h.j1 < g.ny && hh > 0 && ww > 0;
        if (valid && (size_t)hh * ww * sizeof(V) <= lds_bytes - qbytes) {
            st.on = true;
            st.i0 = h.i0;
            st.j0 = h.j0;
            st.h = hh;
            st.w = ww;
            V *dst = reinterpret_cast<V *>(lds + qbytes);
            const V *ev = reinterpret_cast<const V *>(ef);
            const int nodes = hh * ww;
            const int nt = (int)blockDim.x;
            for (int t0 = threadIdx.x; t0 < nodes; t0 += 4 * nt) {
                V v[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int t = t0 + k * nt;
                    const int r = t / ww;
                    v[k] = t < nodes ? ev[(h.i0 + r) * g.ny + h.j0 + (t - r * ww)] : V{};
                }
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (t0 + k * nt < nodes) dst[t0 + k * nt] = v[k];
            }
            le = dst;
        }
    }
    if constexpr (DEPOSIT) {
        uint4 *q4 = reinterpret_cast<uint4 *>(lds_q);
        for (int t = threadIdx.x; t < ncell / 4; t += blockDim.x) q4[t] = make_uint4(0, 0, 0, 0);
        if (threadIdx.x == 0) {
            s_box[0] = INT_MAX;
            s_box[1] = -1;
            s_box[2] = INT_MAX;
            s_box[3] = -1;
            *s_count = 0;
        }
    }
    if (KICK || DEPOSIT) __syncthreads();
    const bool moves = KICK || els.n_el > 0;
    int bi0 = INT_MAX, bi1 = -1, bj0 = INT_MAX, bj1 = -1, cnt = 0;
    for (; p < P.n; p += T) {
        const int64_t pn = p + T;
        double xn = 0, pxn = 0, yn = 0, pyn = 0;
        uint8_t lfn = 1;
        if (pn < P.n) {
            xn = P.x[pn];
            pxn = P.px[pn];
            yn = P.y[pn];
            pyn = P.py[pn];
            lfn = P.lost ? P.lost[pn] : 0;
        }
        bool act = lf == 0;
        if (KICK && act) {
            Cic c;
            if (cic(g, x, y, c)) {
                TE fx, fy;
                const int li = c.i - st.i0, lj = c.j - st.j0;
                if (st.on && li >= 0 && li + 1 < st.h && lj >= 0 && lj + 1 < st.w)
                    gather_lds(le, li * st.w + lj, st.w, c, fx, fy);
                else
                    gather(ef, c.i * g.ny + c.j, g.ny, c, fx, fy);
                px = px + kappa * (double)fx;
                py = py + kappa * (double)fy;
            } else if (P.lost) {
                P.lost[p] = 1;
                act = false;
            }
        }
        if (act) {
            for (int e = 0; e < els.n_el; ++e) apply_element(els.kind[e], els.p[e], x, px, y, py);
            if (moves) {
                P.x[p] = x;
                P.px[p] = px;
                P.y[p] = y;
                P.py[p] = py;
            }
            if constexpr (DEPOSIT) {
                Cic c;
                if (cic(g, x, y, c)) {
                    lds_deposit(lds_q, c.i * g.ny + c.j, g.ny, c, dep.carry);
                    bi0 = min(bi0, c.i);
                    bi1 = max(bi1, c.i + 1);
                    bj0 = min(bj0, c.j);
                    bj1 = max(bj1, c.j + 1);
                    ++cnt;
                } else if (P.lost) {
                    P.lost[p] = 1;
                }
            }
        }
        x = xn;
        px = pxn;
        y = yn;
        py = pyn;
        lf = lfn;
    }
    if constexpr (DEPOSIT) flush_partials(g, dep, lds_q, s_box, s_count, bi0, bi1, bj0, bj1, cnt);
}

// General path: any number of particles per thread, global gathers, the
// charge grid zeroed up front.
template <typename TE, bool KICK, bool DEPOSIT, int U>
__device__ __forceinline__ void pass_batches(const ParticlePtrs &P, const GridGeom &g,
                                             const TE *__restrict__ ef, double kappa,
                                             const PassElements &els, const DepositTarget &dep,
                                             uint32_t *lds_q, int *s_box, int *s_count)
{
    const int ncell = g.nx * g.ny;
    if constexpr (DEPOSIT) {
        uint4 *q4 = reinterpret_cast<uint4 *>(lds_q);
        for (int c = threadIdx.x; c < ncell / 4; c += blockDim.x) q4[c] = make_uint4(0, 0, 0, 0);
        if (threadIdx.x == 0) {
            s_box[0] = INT_MAX;
            s_box[1] = -1;
            s_box[2] = INT_MAX;
            s_box[3] = -1;
            *s_count = 0;
        }
        __syncthreads();
    }
    const bool moves = KICK || els.n_el > 0;
    int bi0 = INT_MAX, bi1 = -1, bj0 = INT_MAX, bj1 = -1, cnt = 0;
    const int64_t T = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; base < P.n;
         base += U * T) {
        double x[U], px[U], y[U], py[U];
        bool act[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t p = base + u * T;
            act[u] = p < P.n;
            uint8_t lf = 0;
            if (act[u]) {
                x[u] = P.x[p];
                px[u] = P.px[p];
                y[u] = P.y[p];
                py[u] = P.py[p];
                if (P.lost) lf = P.lost[p];
            }
            act[u] = act[u] && lf == 0;
        }
        if constexpr (KICK) {
            Cic c[U];
            bool in[U];
            TE fx[U], fy[U];
#pragma unroll
            for (int u = 0; u < U; ++u) in[u] = act[u] && cic(g, x[u], y[u], c[u]);
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (in[u]) gather(ef, c[u].i * g.ny + c[u].j, g.ny, c[u], fx[u], fy[u]);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (in[u]) {
                    px[u] = px[u] + kappa * (double)fx[u];
                    py[u] = py[u] + kappa * (double)fy[u];
                } else if (act[u] && P.lost) {
                    P.lost[base + u * T] = 1;
                    act[u] = false;
                }
            }
        }
        for (int e = 0; e < els.n_el; ++e) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (act[u]) apply_element(els.kind[e], els.p[e], x[u], px[u], y[u], py[u]);
        }
        if (moves) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (!act[u]) continue;
                const int64_t p = base + u * T;
                P.x[p] = x[u];
                P.px[p] = px[u];
                P.y[p] = y[u];
                P.py[p] = py[u];
            }
        }
        if constexpr (DEPOSIT) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (!act[u]) continue;
                Cic c;
                if (cic(g, x[u], y[u], c)) {
                    lds_deposit(lds_q, c.i * g.ny + c.j, g.ny, c, dep.carry);
                    bi0 = min(bi0, c.i);
                    bi1 = max(bi1, c.i + 1);
                    bj0 = min(bj0, c.j);
                    bj1 = max(bj1, c.j + 1);
                    ++cnt;
                } else if (P.lost) {
                    P.lost[base + u * T] = 1;
                }
            }
        }
    }
    if constexpr (DEPOSIT) flush_partials(g, dep, lds_q, s_box, s_count, bi0, bi1, bj0, bj1, cnt);
}

template <typename TE, bool KICK, bool DEPOSIT, int U>
__global__ void __launch_bounds__(1024)
    k_pass(ParticlePtrs P, GridGeom g, const TE *__restrict__ ef, double kappa,
           PassElements els, DepositTarget dep, unsigned lds_bytes, int variant)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ int s_box[4];
    __shared__ int s_count;
    const int64_t T = (int64_t)gridDim.x * blockDim.x;
    if (variant == 1)
        pass_stream<TE, KICK, DEPOSIT>(P, g, ef, kappa, els, dep, lds_raw, lds_bytes, s_box,
                                       &s_count);
    else if ((KICK || DEPOSIT) && (int64_t)U * T >= P.n)
        pass_single_batch<TE, KICK, DEPOSIT, U>(P, g, ef, kappa, els, dep, lds_raw, lds_bytes,
                                                s_box, &s_count);
    else
        pass_batches<TE, KICK, DEPOSIT, U>(P, g, ef, kappa, els, dep,
                                           reinterpret_cast<uint32_t *>(lds_raw), s_box, &s_count);
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

constexpr int kUnroll = 4;

// Dynamic LDS of a pass launch: the charge grid for a depositing pass, and
// for a kicking pass room for the staged field box, up to the workgroup limit.
size_t pass_lds_bytes(bool kick, bool deposit, int ncell, size_t lds_limit)
{
    size_t b = deposit ? sizeof(uint32_t) * (size_t)ncell : 0;
    if (kick) b = std::max(b, lds_limit);
    return b;
}

size_t g_lds_limit = 0;  // set by prepare_pass_kernels

template <typename TE, bool KICK, bool DEPOSIT>
hipError_t launch_pass_t(hipStream_t s, const ParticlePtrs &p, const GridGeom &g, const void *ef,
                         double kappa, const PassElements &els, const DepositTarget &dep,
                         int blocks, int threads, int variant)
{
    const size_t lds = pass_lds_bytes(KICK, DEPOSIT, g.nx * g.ny, g_lds_limit);
    hipLaunchKernelGGL((k_pass<TE, KICK, DEPOSIT, kUnroll>), dim3(blocks), dim3(threads), lds, s,
                       p, g, (const TE *)ef, kappa, els, dep, (unsigned)lds, variant);
    return hipGetLastError();
}

}  // namespace

// Allow the passes the dynamic LDS they use (beyond the default limit):
// lds_limit is the device's per-workgroup LDS minus the kernel's static LDS.
// Called once per context, outside any stream capture.
hipError_t prepare_pass_kernels(size_t lds_limit)
{
    g_lds_limit = lds_limit;
    const void *kerns[] = {(const void *)k_pass<double, true, true, kUnroll>,
                           (const void *)k_pass<double, false, true, kUnroll>,
                           (const void *)k_pass<double, true, false, kUnroll>,
                           (const void *)k_pass<float, true, true, kUnroll>,
                           (const void *)k_pass<float, false, true, kUnroll>,
                           (const void *)k_pass<float, true, false, kUnroll>};
    for (const void *k : kerns) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds_limit);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_pass(hipStream_t s, const ParticlePtrs &p, const GridGeom &g, bool kick,
                       bool mixed, const void *ef, double kappa, const PassElements &els,
                       bool deposit, const DepositTarget &dep, int blocks, int threads,
                       int variant)
{
    if (blocks <= 0) return hipSuccess;
    if (mixed) {
        if (kick)
            return deposit ? launch_pass_t<float, true, true>(s, p, g, ef, kappa, els, dep, blocks, threads, variant)
                           : launch_pass_t<float, true, false>(s, p, g, ef, kappa, els, dep, blocks, threads, variant);
        return deposit ? launch_pass_t<float, false, true>(s, p, g, ef, kappa, els, dep, blocks, threads, variant)
                       : launch_pass_t<float, false, false>(s, p, g, ef, kappa, els, dep, blocks, threads, variant);
    }
    if (kick)
        return deposit ? launch_pass_t<double, true, true>(s, p, g, ef, kappa, els, dep, blocks, threads, variant)
                       : launch_pass_t<double, true, false>(s, p, g, ef, kappa, els, dep, blocks, threads, variant);
    return deposit ? launch_pass_t<double, false, true>(s, p, g, ef, kappa, els, dep, blocks, threads, variant)
                   : launch_pass_t<double, false, false>(s, p, g, ef, kappa, els, dep, blocks, threads, variant);
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
