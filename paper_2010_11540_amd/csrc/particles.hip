// Particle-side kernels of libscpic for gfx950: the fused particle pass
// (gather + kick, push, cloud-in-cell deposit into LDS) and the reduction of
// the per-block charge partials.
//
// Compiled with -ffp-contract=off: every FP64 expression below is evaluated
// as written, each operation correctly rounded, so the cell index, the
// fixed-point weights and a linear push are bit-identical to the same IEEE
// sums evaluated anywhere else.
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

// The fused particle pass.  Thread t of the launch (T threads in all) takes
// the particles t + u*T + k*U*T, u < U: consecutive lanes take consecutive
// particles, so every SoA load and store is coalesced, and each thread issues
// the loads of its U particles before using any, so U particles per lane are
// in flight at once.  For each particle:
//   KICK     gather the node field at the particle with the deposit weights
//            and kick px, py by kappa * E (a particle found outside the domain
//            is marked lost and frozen);
//   push     through els (uniform, read from the kernel arguments);
//   DEPOSIT  add the particle's four weights to the workgroup's private copy
//            of the charge grid in LDS (particles outside are marked lost).
// At the end each workgroup writes the bounding box of the cells it touched,
// packed densely, to its own slice of the partials (no global atomics).
template <typename TE, bool KICK, bool DEPOSIT, int U>
__global__ void __launch_bounds__(1024)
    k_pass(ParticlePtrs P, GridGeom g, const TE *__restrict__ ef, double kappa,
           PassElements els, DepositTarget dep)
{
    extern __shared__ uint32_t lds_q[];
    __shared__ int s_box[4];
    __shared__ int s_count;
    const int ncell = g.nx * g.ny;
    if constexpr (DEPOSIT) {
        uint4 *q4 = reinterpret_cast<uint4 *>(lds_q);
        for (int c = threadIdx.x; c < ncell / 4; c += blockDim.x) q4[c] = make_uint4(0, 0, 0, 0);
        if (threadIdx.x == 0) {
            s_box[0] = INT_MAX;
            s_box[1] = -1;
            s_box[2] = INT_MAX;
            s_box[3] = -1;
            s_count = 0;
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
    }
    if constexpr (DEPOSIT) {
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
        const int i0 = s_box[0], i1 = s_box[1], j0 = s_box[2], j1 = s_box[3];
        uint32_t *out = dep.partial + (size_t)blockIdx.x * ncell;
        if (i0 <= i1) {
            const int w = j1 - j0 + 1;
            const int total = (i1 - i0 + 1) * w;
            for (int t = threadIdx.x; t < total; t += blockDim.x) {
                const int r = t / w;
                out[t] = lds_q[(i0 + r) * g.ny + j0 + (t - r * w)];
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
            dep.header[blockIdx.x] = h;
        }
    }
}

// Exact charge grid q = sum over workgroups of their partials (+ carries).
// The block headers are staged in LDS first; then a workgroup owns 64
// consecutive cells (one per lane) and its 16 waves split the partials, so
// every partial load of a lane is independent and in flight together; the
// per-wave sums are combined in LDS.  The carry grid is consumed and cleared.
constexpr int kReduceWaves = 16;

__global__ void __launch_bounds__(kReduceWaves * 64)
    k_reduce(DepositTarget dep, int nblocks, int nx, int ny, int64_t *__restrict__ q,
             int64_t *__restrict__ n_in)
{
    __shared__ BlockHeader hdr[kMaxPassBlocks];
    __shared__ unsigned long long part[kReduceWaves][64];
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) hdr[b] = dep.header[b];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ncell = nx * ny;
    const int c = blockIdx.x * 64 + lane;
    const int i = c / ny, j = c - i * ny;
    unsigned long long s = 0;
#pragma unroll 8
    for (int b = wave; b < nblocks; b += kReduceWaves) {
        const BlockHeader h = hdr[b];
        if (i >= h.i0 && i <= h.i1 && j >= h.j0 && j <= h.j1) {
            const int w = h.j1 - h.j0 + 1;
            s += dep.partial[(size_t)b * ncell + (i - h.i0) * w + (j - h.j0)];
        }
    }
    part[wave][lane] = s;
    __syncthreads();
    if (wave == 0) {
        unsigned long long t = 0;
#pragma unroll
        for (int k = 0; k < kReduceWaves; ++k) t += part[k][lane];
        t += dep.carry[c];
        dep.carry[c] = 0ull;
        q[c] = (int64_t)t;
    }
    if (n_in != nullptr && blockIdx.x == 0 && wave == 1) {
        long long cnt = 0;
        for (int b = lane; b < nblocks; b += 64) cnt += hdr[b].count;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
        if (lane == 0) *n_in = cnt;
    }
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

template <typename TE, bool KICK, bool DEPOSIT>
hipError_t launch_pass_t(hipStream_t s, const ParticlePtrs &p, const GridGeom &g, const void *ef,
                         double kappa, const PassElements &els, const DepositTarget &dep,
                         int blocks, int threads)
{
    const size_t lds = DEPOSIT ? sizeof(uint32_t) * (size_t)g.nx * g.ny : 0;
    hipLaunchKernelGGL((k_pass<TE, KICK, DEPOSIT, kUnroll>), dim3(blocks), dim3(threads), lds, s,
                       p, g, (const TE *)ef, kappa, els, dep);
    return hipGetLastError();
}

}  // namespace

// Allow the depositing passes the dynamic LDS of a whole charge grid (up to
// 64 KiB, beyond the default limit); called once per context, outside any
// stream capture.
hipError_t prepare_pass_kernels(size_t lds_bytes)
{
    const void *kerns[] = {(const void *)k_pass<double, true, true, kUnroll>,
                           (const void *)k_pass<double, false, true, kUnroll>,
                           (const void *)k_pass<float, true, true, kUnroll>,
                           (const void *)k_pass<float, false, true, kUnroll>};
    for (const void *k : kerns) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_pass(hipStream_t s, const ParticlePtrs &p, const GridGeom &g, bool kick,
                       bool mixed, const void *ef, double kappa, const PassElements &els,
                       bool deposit, const DepositTarget &dep, int blocks, int threads)
{
    if (blocks <= 0) return hipSuccess;
    if (mixed) {
        if (kick)
            return deposit ? launch_pass_t<float, true, true>(s, p, g, ef, kappa, els, dep, blocks, threads)
                           : launch_pass_t<float, true, false>(s, p, g, ef, kappa, els, dep, blocks, threads);
        return deposit ? launch_pass_t<float, false, true>(s, p, g, ef, kappa, els, dep, blocks, threads)
                       : launch_pass_t<float, false, false>(s, p, g, ef, kappa, els, dep, blocks, threads);
    }
    if (kick)
        return deposit ? launch_pass_t<double, true, true>(s, p, g, ef, kappa, els, dep, blocks, threads)
                       : launch_pass_t<double, true, false>(s, p, g, ef, kappa, els, dep, blocks, threads);
    return deposit ? launch_pass_t<double, false, true>(s, p, g, ef, kappa, els, dep, blocks, threads)
                   : launch_pass_t<double, false, false>(s, p, g, ef, kappa, els, dep, blocks, threads);
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

hipError_t launch_reduce(hipStream_t s, const DepositTarget &dep, int blocks_used, int nx, int ny,
                         int64_t *q, int64_t *n_in)
{
    const int ncell = nx * ny;  // a multiple of 64 for every supported grid
    hipLaunchKernelGGL(k_reduce, dim3(ncell / 64), dim3(kReduceWaves * 64), 0, s, dep, blocks_used,
                       nx, ny, q, n_in);
    return hipGetLastError();
}

}  // namespace scpic
