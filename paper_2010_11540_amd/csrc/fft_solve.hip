// Grid-side kernels of libscpic for gfx950: the exact reduction of the
// per-workgroup charge partials and the open-boundary Poisson solve as a
// zero-padded FFT convolution with the free-space Green's function (Hockney's
// method), the centred-difference field taken in the spectrum.  Each axis is
// padded to the power of two mx >= 2 nx (my >= 2 ny): any such length makes
// the cyclic convolution equal the linear one on nodes -1..n.  Hand-written
// radix-4/2 Stockham FFTs in LDS, each run by one wave, reading per-stage
// twiddle tables and XOR-swizzled buffers so that no stage's LDS accesses
// conflict on banks; no vendor FFT library.
//
// Data flow for a charge grid q (nx x ny, rows i along x; hy = my / 2):
//   k_rows_fwd   one workgroup per row i: sum the row's partials exactly
//                (uint64, + carries) or read a dense int64 row, scale to
//                rho; the real row zero-padded to my is transformed as a
//                complex FFT of half length hy (even/odd samples packed) and
//                untangled into the half spectrum l = 0..hy   -> A^T [hy+1][nx]
//   k_cols       per column l: FFT along x (length mx, zero-padded),
//                multiply by the real Green's spectrum G^(k,l) (inverse-FFT
//                normalisation folded in), then two inverse FFTs run by two
//                waves at once: -i sin(2 pi k/mx)/dx * Phi (the x central
//                difference) and Phi, scaled by -i sin(2 pi l/my)/dy (the y
//                central difference); rows 0..nx-1 kept -> Bx, By [nx][hy+1]
//   k_rows_inv   per row i: both half spectra packed as Ex + i Ey, completed
//                by Hermitian symmetry, one inverse FFT     -> ex, ey [nx][ny]
// Taking the differences in the spectrum keeps the large constant part of
// the potential out of the field's rounding, which matters for the FP32 form.
// Every kernel issues all of its global loads into registers before the
// first LDS write, so each kernel waits for one round of memory latency.
#include <algorithm>

#include "scpic_internal.h"

// The solve carries no bit-exactness contract (its field is compared with the
// direct-sum solve within a tolerance, and the batched and single-beam paths
// share this code): multiply-adds may be fused here, unlike in the pass.
#pragma clang fp contract(fast)

namespace scpic {
namespace {

template <typename T>
struct cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
template <typename T>
__device__ __forceinline__ cx<T> scale_c(cx<T> a, T s) { return {a.re * s, a.im * s}; }
// -i * a
template <typename T>
__device__ __forceinline__ cx<T> mul_neg_i(cx<T> a) { return {a.im, -a.re}; }
// +i * a
template <typename T>
__device__ __forceinline__ cx<T> mul_pos_i(cx<T> a) { return {-a.im, a.re}; }

// Orders one wave's LDS accesses across an FFT stage: a wave's LDS
// instructions execute in order, so the fences only stop the compiler from
// moving a read of the next stage above a write of this one.
__device__ __forceinline__ void wave_lds_order()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS slot of element e of an FFT buffer: e with bits 0-4 XORed by bits 2-6
// (a permutation within each aligned block of 32 elements, and of any
// shorter buffer).  With it the strided writes of the early FFT stages (and
// their reads) fall on distinct banks, which the natural order does not:
// there a stage's outputs are written 4 ns elements apart per lane.
__device__ __forceinline__ int sw(int e) { return e ^ ((e >> 2) & 31); }

// Forward DFT X[k] = sum_n x[n] exp(-2 pi i n k / L) of the sequence in LDS
// buffer a (length L = 2^log2L), ping-ponging with buffer b, computed by ONE
// wave: lane = 0..63 of that wave (a lane index >= L/2 takes no butterfly,
// which lets the other waves of a workgroup call it too, as a no-op).  The
// input must be visible to the wave when it is called (a workgroup barrier if
// other waves wrote it); the result is visible to the same wave on return and
// to the others after a workgroup barrier.  Stockham autosort: one radix-2
// stage first when log2L is odd, then radix-4 stages; each stage reads
// sub-transform inputs L/r apart, applies the twiddles exp(-2 pi i m k / (Ns r))
// and writes the r outputs Ns apart.  st: the stage twiddles of an L-point
// FFT (stage_twiddle_count), in LDS.
// Returns the buffer holding X in natural order (the same in every lane).
template <typename T>
__device__ cx<T> *fft_wave(cx<T> *a, cx<T> *b, int L, int log2L, const cx<T> *st, int lane)
{
    int ns = 1;
    if (log2L & 1) {
        const int h = L >> 1;
        for (int j = lane; j < h; j += 64) {
            const cx<T> u = a[sw(j)], v = a[sw(j + h)];
            b[sw(2 * j)] = u + v;
            b[sw(2 * j + 1)] = u - v;
        }
        cx<T> *t = a;
        a = b;
        b = t;
        ns = 2;
        wave_lds_order();
    }
    const int c = ns;
    const int q = L >> 2;
    while (ns < L) {
        const cx<T> *ws = st + (ns - c);
        for (int j = lane; j < q; j += 64) {
            const int k = j & (ns - 1);
            const cx<T> *w = ws + 3 * k;
            const cx<T> a0 = a[sw(j)];
            const cx<T> a1 = cmul(a[sw(j + q)], w[0]);
            const cx<T> a2 = cmul(a[sw(j + 2 * q)], w[1]);
            const cx<T> a3 = cmul(a[sw(j + 3 * q)], w[2]);
            const cx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = a1 - a3;
            const int base = (j - k) * 4 + k;
            b[sw(base)] = t0 + t2;
            b[sw(base + ns)] = t1 + mul_neg_i(t3);
            b[sw(base + 2 * ns)] = t0 - t2;
            b[sw(base + 3 * ns)] = t1 + mul_pos_i(t3);
        }
        cx<T> *t = a;
        a = b;
        b = t;
        ns *= 4;
        wave_lds_order();
    }
    return a;
}

constexpr int kRowThreads = 1024;  // row-forward: 16 waves share the reduction
constexpr int kColThreads = 256;   // columns: 4 waves; waves 0 and 1 run the inverse transforms
constexpr int kInvThreads = 256;   // row-inverse: loads and stores over 4 waves
constexpr int kMaxPerThread = kMaxFft / 64;

// Exact sum of grid row i over the partials of nblocks workgroups plus the
// carry grid (which is cleared), for the ny cells of the row.  Called by all
// NT threads of the workgroup (NT >= ny).  Thread t reads 16-byte chunks (4 cells) of the row:
// ny/4 lanes cover one workgroup's row segment and the kRowThreads/(ny/4)
// groups of lanes split the workgroups, each issuing all of its loads before
// adding any (one round of memory latency for <= kReduceChunk workgroups per
// lane).  Chunks outside a workgroup's bounding box are not read (their
// loads return zeros without touching memory).  hdr: the headers staged in LDS; red: LDS
// scratch of NT * 4 uint64; carry_v: this cell's carry, loaded by
// the caller with its first round of loads (cleared here when nonzero).
// Returns the total of cell tid (tid < ny).
constexpr int kReduceChunk = 8;

// Lane layout of a row reduction by NT threads: lanes = ny/4 16-byte chunks
// cover one workgroup's row segment (ny is a multiple of 4), and groups =
// NT/lanes whole groups of lanes split the workgroups.
struct RowLanes {
    int lanes, groups, grp, j0c;
};
template <int NT>
__device__ __forceinline__ RowLanes row_lanes(int ny, int tid)
{
    RowLanes r;
    r.lanes = ny >> 2;
    r.groups = NT / r.lanes;  // ny <= 256 -> at least NT / 64
    r.grp = tid / r.lanes;
    r.j0c = (tid - r.grp * r.lanes) * 4;
    return r;
}

template <int NT>
__device__ __forceinline__ unsigned long long reduce_row(const DepositTarget &dep,
                                                         const BlockHeader *hdr,
                                                         unsigned long long *red, int nblocks,
                                                         int i, int ny, int tid,
                                                         unsigned long long carry_v)
{
    const RowLanes L = row_lanes<NT>(ny, tid);
    const int groups = L.groups, grp = L.grp, j0c = L.j0c;
    // when ny / 4 does not divide NT the last threads form no whole group
    const bool member = grp < groups;
    // The partials as a buffer: a chunk outside a workgroup's box is read at
    // an offset past the buffer's end, which returns zeros and touches no
    // memory.  A chunk inside the box holds the box's cells and zeros (the
    // tile's cells outside the box are zero), so no cell needs a mask.
    const uint32_t bytes = (uint32_t)(sizeof(uint32_t) * (size_t)dep.max_blocks * ny) *
                           (uint32_t)(i + 1);
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(dep.partial, (short)0, (int)bytes, 0x00020000);
    constexpr uint32_t kOutside = 0x80000000u;
    const uint32_t row0 = (uint32_t)(sizeof(uint32_t) * ((size_t)i * dep.max_blocks * ny + j0c));
    unsigned long long s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int b0 = member ? grp : nblocks; b0 < nblocks; b0 += groups * kReduceChunk) {
        uint32_t off[kReduceChunk];
#pragma unroll
        for (int u = 0; u < kReduceChunk; ++u) {
            const int b = b0 + u * groups;
            const BlockHeader h = hdr[b < nblocks ? b : 0];
            const bool take = b < nblocks && i >= h.i0 && i <= h.i1 && j0c + 3 >= h.j0 &&
                              j0c <= h.j1;
            off[u] = take ? row0 + (uint32_t)(sizeof(uint32_t) * (size_t)b * ny) : kOutside;
        }
        // every load in flight before the first add
        decltype(__builtin_amdgcn_raw_buffer_load_b128(rs, 0, 0, 0)) v[kReduceChunk];
#pragma unroll
        for (int u = 0; u < kReduceChunk; ++u)
            v[u] = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off[u], 0, 0);
#pragma unroll
        for (int u = 0; u < kReduceChunk; ++u) {
            s0 += (uint32_t)v[u][0];
            s1 += (uint32_t)v[u][1];
            s2 += (uint32_t)v[u][2];
            s3 += (uint32_t)v[u][3];
        }
    }
    if (member) {
        unsigned long long *mine = red + (size_t)grp * ny + j0c;
        mine[0] = s0;
        mine[1] = s1;
        mine[2] = s2;
        mine[3] = s3;
    }
    __syncthreads();
    unsigned long long t = 0;
    if (tid < ny) {
        for (int g = 0; g < groups; ++g) t += red[(size_t)g * ny + tid];
        t += carry_v;
        if (carry_v) dep.carry[(size_t)i * ny + tid] = 0ull;
    }
    return t;
}

// Exact int64 charge grid (scpic_deposit): one workgroup per row.
__global__ void __launch_bounds__(kRowThreads)
    k_reduce(DepositTarget dep, int nblocks, int nx, int ny, int64_t *__restrict__ q,
             int64_t *__restrict__ n_in)
{
    __shared__ BlockHeader hdr[kMaxPassBlocks];
    __shared__ unsigned long long red[kRowThreads * 4];
    const int tid = threadIdx.x, i = blockIdx.x;
    const unsigned long long cv = tid < ny ? dep.carry[(size_t)i * ny + tid] : 0ull;
    for (int b = tid; b < nblocks; b += kRowThreads) hdr[b] = dep.header[b];
    __syncthreads();
    const unsigned long long t = reduce_row<kRowThreads>(dep, hdr, red, nblocks, i, ny, tid, cv);
    if (tid < ny) q[(size_t)i * ny + tid] = (int64_t)t;
    if (n_in != nullptr && i == 0 && tid < 64) {
        long long cnt = 0;
        for (int b = tid; b < nblocks; b += 64) cnt += hdr[b].count;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
        if (tid == 0) *n_in = cnt;
    }
}

// Row i of rho (from the partials when FROM_PARTIALS, else from a dense int64
// grid), real and zero-padded to my = 2 hy: packed z[m] = rho[2m] + i rho[2m+1]
// (zero from index ny on), Z = FFT_hy(z), then
//   X[l] = (Z[l] + conj Z[hy-l]) / 2 - i W^l (Z[l] - conj Z[hy-l]) / 2,
// W = exp(-2 pi i / my), for l = 0..hy.  tw: W^l for l = 0..hy, then the
// stage twiddles of the hy-point FFT (the grid's stw_y table).
// LDS of the row-forward workgroup: the twiddles W^l, l = 0..hy, the stage
// twiddles of the hy-point FFT [hy], two FFT buffers [hy], rho [ny], then
// (16-byte aligned) the staged headers.
template <typename T>
__host__ __device__ constexpr size_t rows_fwd_hdr_offset(int ny, int my)
{
    return (sizeof(cx<T>) * (size_t)(2 * my + 1) + sizeof(T) * (size_t)ny + 15) & ~(size_t)15;
}

template <typename T, bool FROM_PARTIALS, int NT>
__device__ __forceinline__ void rows_fwd_body(const DepositTarget &dep, int nblocks,
                                              const int64_t *__restrict__ q, double scale, int nx,
                                              int ny, int my, int log2my,
                                              const cx<T> *__restrict__ tw, cx<T> *__restrict__ at,
                                              int i, bool pipe)
{
    extern __shared__ unsigned char smem_raw[];
    const int half = my >> 1;                           // hy: complex FFT length
    cx<T> *twl = reinterpret_cast<cx<T> *>(smem_raw);  // W^l, l = 0..hy
    cx<T> *st = twl + half + 1;                         // stage twiddles, hy
    cx<T> *a = st + half;                               // hy
    cx<T> *b = a + half;                                // hy
    T *rho = reinterpret_cast<T *>(b + half);           // ny
    BlockHeader *hdr = reinterpret_cast<BlockHeader *>(smem_raw + rows_fwd_hdr_offset<T>(ny, my));
    __shared__ unsigned long long red[FROM_PARTIALS ? NT * 4 : 1];
    const int tid = threadIdx.x;
    // one round of loads: twiddles, and the headers or the dense row (ny <= NT)
    const int64_t qv = (!FROM_PARTIALS && tid < ny) ? q[(size_t)i * ny + tid] : 0;
    const unsigned long long cv =
        (FROM_PARTIALS && tid < ny) ? dep.carry[(size_t)i * ny + tid] : 0ull;
    // W^l for l <= hy and the hy-point FFT's stage twiddles, as stored
    for (int t = tid; t <= half + stage_twiddle_count(half, log2my - 1); t += NT) twl[t] = tw[t];
    if (FROM_PARTIALS)
        for (int t = tid; t < nblocks; t += NT) hdr[t] = dep.header[t];
    if (FROM_PARTIALS) {
        __syncthreads();
        const unsigned long long t = reduce_row<NT>(dep, hdr, red, nblocks, i, ny, tid, cv);
        if (tid < ny) rho[tid] = (T)((double)t * scale);
    } else {
        if (tid < ny) rho[tid] = (T)((double)qv * scale);
    }
    __syncthreads();
    // the row as a real sequence of length my: zero-padded (open boundary),
    // or odd-extended about the walls at j = 0 and j = ny (grounded pipe; the
    // wall row i = 0 and the wall column j = 0 take no charge)
    auto sample = [&](int l) -> T {
        if (!pipe) return l < ny ? rho[l] : T(0);
        if (i == 0 || l == 0 || l == ny) return T(0);
        return l < ny ? rho[l] : -rho[my - l];
    };
    if (tid < half) a[sw(tid)] = cx<T>{sample(2 * tid), sample(2 * tid + 1)};
    __syncthreads();
    // wave 0 transforms; the other waves only learn where the result lies
    const cx<T> *Z = fft_wave(a, b, half, log2my - 1, st, tid < 64 ? tid : half);
    __syncthreads();
    for (int l = tid; l <= half; l += NT) {
        const cx<T> zl = Z[sw(l & (half - 1))];
        const cx<T> zm = conj(Z[sw((half - l) & (half - 1))]);
        const cx<T> s = zl + zm, d = zl - zm;
        const cx<T> wd = mul_neg_i(cmul(twl[l], d));
        at[(size_t)l * nx + i] = scale_c(s + wd, T(0.5));
    }
}

// Line density of a long bunch (Sec. IV): sum the nblocks per-workgroup
// histograms of the last depositing pass exactly and write the node tables
//   lw[k] = h[k] / max h,   ld[k] = (h[k+1] - h[k-1]) / (2 dz max h)
// (h = 0 beyond the line; all zero for an empty line).  NT / nz groups of
// threads split the workgroups; acc is NT words of dynamic LDS.
template <int NT>
__device__ __forceinline__ void line_table_body(const LineSpec &L, int nblocks)
{
    extern __shared__ unsigned char smem_raw[];
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(smem_raw);
    __shared__ unsigned long long wmax[NT / 64];
    const int tid = threadIdx.x, nz = L.nz;
    const int groups = NT / nz;
    const int k = tid % nz, g = tid / nz;
    unsigned long long s = 0;
    if (g < groups)
        for (int b0 = g; b0 < nblocks; b0 += 8 * groups) {
            unsigned long long v[8];  // eight loads in flight per round
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int b = b0 + u * groups;
                v[u] = b < nblocks ? L.partial[(size_t)b * nz + k] : 0ull;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
    acc[tid] = s;
    __syncthreads();
    unsigned long long h = 0;
    if (tid < nz)
        for (int r = 0; r < groups; ++r) h += acc[r * nz + tid];
    __syncthreads();
    if (tid < nz) acc[tid] = h;
    unsigned long long m = h;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long v = __shfl_xor(m, o, 64);
        m = v > m ? v : m;
    }
    if ((tid & 63) == 0) wmax[tid >> 6] = m;
    __syncthreads();
    unsigned long long hmax = 0;
    for (int w = 0; w < NT / 64; ++w) hmax = wmax[w] > hmax ? wmax[w] : hmax;
    if (tid < nz) {
        double lw = 0.0, ld = 0.0;
        if (hmax) {
            const long long up = tid + 1 < nz ? (long long)acc[tid + 1] : 0;
            const long long down = tid > 0 ? (long long)acc[tid - 1] : 0;
            lw = (double)h / (double)hmax;
            ld = (double)(up - down) / (2.0 * L.dz * (double)hmax);
        }
        L.lw[tid] = lw;
        L.ld[tid] = ld;
    }
}

// Rows of the charge grid; with a line density (line.nz > 0) one more
// workgroup, index nx, reduces the line histograms.
template <typename T, bool FROM_PARTIALS>
__global__ void __launch_bounds__(kRowThreads)
    k_rows_fwd(DepositTarget dep, int nblocks, const int64_t *__restrict__ q, double scale,
               int nx, int ny, int my, int log2my, const cx<T> *__restrict__ tw,
               cx<T> *__restrict__ at, bool pipe, LineSpec line)
{
    if (line.nz > 0 && (int)blockIdx.x == nx) {
        line_table_body<kRowThreads>(line, nblocks);
        return;
    }
    rows_fwd_body<T, FROM_PARTIALS, kRowThreads>(dep, nblocks, q, scale, nx, ny, my, log2my, tw,
                                                 at, (int)blockIdx.x, pipe);
}

// Every beam of a batch: workgroup -> (beam, row) from the batch's row table;
// the rows come from the partials of the beam's last batched pass.  A beam's
// row has few partial slices, so a smaller workgroup does it and more of them
// fit on a compute unit at once: NT threads, at least the largest ny and hy
// of the batch (128 when every beam's grid has ny <= 128, else 256).
template <typename T, int NT>
__global__ void __launch_bounds__(NT) k_rows_fwd_batched(BatchLaunch b)
{
    const BatchInstance &I = b.inst[b.row_inst[blockIdx.x]];
    rows_fwd_body<T, true, NT>(I.dep, I.pass_blocks, nullptr, I.scale, I.nx, I.ny,
                                             I.my, I.log2_my, (const cx<T> *)I.stw_y,
                                             (cx<T> *)I.spec_a, (int)blockIdx.x - I.row_block0,
                                             false);
}

// Column l (of hy + 1) of the row spectra: forward FFT along x, times the
// Green's spectrum, then the two differentiated inverse transforms, one per
// wave.  The second is the column-inverse of the potential's spectrum before
// the y difference (tw: the stage twiddles of the mx-point FFT); bp, when
// not null, receives it as well for the node
// potential, on rows -1..nx (row i at bp[(i + 1) * (hy + 1)]; row -1 is the
// periodic row mx - 1, which the zero padding or the odd extension makes the
// potential's value one node outside the grid).
template <typename T>
__device__ __forceinline__ void cols_body(const cx<T> *__restrict__ at, int nx, int hy, int mx,
                                          int log2mx, const cx<T> *__restrict__ tw,
                                          const T *__restrict__ ghat_t, const T *__restrict__ sx,
                                          const T *__restrict__ sy, cx<T> *__restrict__ bx,
                                          cx<T> *__restrict__ by, int l, bool pipe,
                                          cx<T> *__restrict__ bp = nullptr)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T> *st = reinterpret_cast<cx<T> *>(smem_raw);  // stage twiddles
    cx<T> *a = st + mx;
    cx<T> *b = a + mx;
    cx<T> *c = b + mx;
    cx<T> *d = c + mx;
    const int tid = threadIdx.x;
    const cx<T> *col = at + (size_t)l * nx;
    const T *g = ghat_t + (size_t)l * mx;
    constexpr int kPer = kMaxFft / kColThreads;
    // every input of the column in one round of loads
    cx<T> vt[kPer], va[kPer];
    T vg[kPer], vs[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int k = tid + r * kColThreads;
        vt[r] = k < stage_twiddle_count(mx, log2mx) ? tw[k] : cx<T>{T(0), T(0)};
        vg[r] = k < mx ? g[k] : T(0);
        vs[r] = k < mx ? sx[k] : T(0);
        // zero-padded column (open boundary), or its odd extension about
        // the walls at i = 0 and i = nx (grounded pipe)
        const int src = k < nx ? k : mx - k;
        const bool zero = pipe ? (k == 0 || k == nx) : k >= nx;
        const cx<T> c = zero ? cx<T>{T(0), T(0)} : col[src];
        va[r] = (pipe && k > nx) ? cx<T>{-c.re, -c.im} : c;
    }
    const T syl = sy[l];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int k = tid + r * kColThreads;
        if (k < mx) {
            st[k] = vt[r];
            a[sw(k)] = va[r];
        }
    }
    __syncthreads();
    const cx<T> *r0 = fft_wave(a, b, mx, log2mx, st, tid < 64 ? tid : mx);
    __syncthreads();
    // Inverse transforms as conj(FFT(conj(.))): stage the conjugated inputs,
    // x difference in c, y part in d.
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int k = tid + r * kColThreads;
        if (k < mx) {
            const cx<T> phi = scale_c(r0[sw(k)], vg[r]);
            c[sw(k)] = conj(mul_neg_i(scale_c(phi, vs[r])));
            d[sw(k)] = conj(phi);
        }
    }
    const int wave = tid >> 6, lane = tid & 63;
    __syncthreads();
    // waves 0 and 1 run the two inverse transforms side by side; waves 2 and
    // 3 only helped load and stage
    if (wave >= 2) return;
    cx<T> *in = wave ? d : c;
    cx<T> *tmp = wave ? b : a;
    const cx<T> *res = fft_wave(in, tmp, mx, log2mx, st, lane);
    if (wave == 0) {
        for (int i = lane; i < nx; i += 64) bx[(size_t)i * (hy + 1) + l] = conj(res[sw(i)]);
    } else if (wave == 1) {
        for (int i = lane; i < nx; i += 64)
            by[(size_t)i * (hy + 1) + l] = mul_neg_i(scale_c(conj(res[sw(i)]), syl));
        if (bp)
            for (int i = lane - 1; i <= nx; i += 64)
                bp[(size_t)(i + 1) * (hy + 1) + l] = conj(res[sw(i < 0 ? mx - 1 : i)]);
    }
}

template <typename T>
__global__ void __launch_bounds__(kColThreads)
    k_cols(const cx<T> *__restrict__ at, int nx, int hy, int mx, int log2mx,
           const cx<T> *__restrict__ tw, const T *__restrict__ ghat_t, const T *__restrict__ sx,
           const T *__restrict__ sy, cx<T> *__restrict__ bx, cx<T> *__restrict__ by, bool pipe,
           cx<T> *__restrict__ bp)
{
    cols_body<T>(at, nx, hy, mx, log2mx, tw, ghat_t, sx, sy, bx, by, (int)blockIdx.x, pipe, bp);
}

template <typename T>
__global__ void __launch_bounds__(kColThreads) k_cols_batched(BatchLaunch b)
{
    const BatchInstance &I = b.inst[b.col_inst[blockIdx.x]];
    cols_body<T>((const cx<T> *)I.spec_a, I.nx, I.my >> 1, I.mx, I.log2_mx, (const cx<T> *)I.stw_x,
                 (const T *)I.ghat_t, (const T *)I.sx, (const T *)I.sy, (cx<T> *)I.spec_bx,
                 (cx<T> *)I.spec_by, (int)blockIdx.x - I.col_block0, false);
}

// Row i: Z[l] = Bx[l] + i By[l] for l = 0..hy and Z[my-l] = conj(Bx[l]) +
// i conj(By[l]) for 0 < l < hy (hy = my / 2); one inverse FFT gives ex + i ey
// on the first ny entries (tw: the stage twiddles of the my-point FFT).  Written
// either as two arrays (ex, ey) or interleaved into ef (Ex, Ey per node).
// With bp (the potential's column-inverse spectrum), a second inverse FFT of
// its Hermitian row writes row i of the node potential phi on columns
// -1..ny (phi[(i + 1) * (ny + 2) + j + 1]); rows -1 and nx (i < 0 or
// i == nx) write only that.
template <typename T>
__device__ __forceinline__ void rows_inv_body(const cx<T> *__restrict__ bx,
                                              const cx<T> *__restrict__ by, int nx, int ny, int my,
                                              int log2my, const cx<T> *__restrict__ tw,
                                              T *__restrict__ ex, T *__restrict__ ey,
                                              cx<T> *__restrict__ ef, int i,
                                              const cx<T> *__restrict__ bp = nullptr,
                                              T *__restrict__ phi = nullptr)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T> *st = reinterpret_cast<cx<T> *>(smem_raw);  // stage twiddles
    cx<T> *a = st + my;
    cx<T> *b = a + my;
    const int tid = threadIdx.x;
    const int hy = my >> 1;
    // rows -1 and nx have no field: their (unused) spectrum loads read row 0
    const int fi = (i >= 0 && i < nx) ? i : 0;
    const cx<T> *rx = bx + (size_t)fi * (hy + 1);
    const cx<T> *ry = by + (size_t)fi * (hy + 1);
    constexpr int kPerT = kMaxFft / kInvThreads;          // twiddles per thread
    constexpr int kPerL = kMaxFft / 2 / kInvThreads + 1;  // spectrum entries per thread
    cx<T> vt[kPerT], vx[kPerL], vy[kPerL];
#pragma unroll
    for (int r = 0; r < kPerT; ++r) {
        const int t = tid + r * kInvThreads;
        vt[r] = t < stage_twiddle_count(my, log2my) ? tw[t] : cx<T>{T(0), T(0)};
    }
#pragma unroll
    for (int r = 0; r < kPerL; ++r) {
        const int l = tid + r * kInvThreads;
        vx[r] = l <= hy ? rx[l] : cx<T>{T(0), T(0)};
        vy[r] = l <= hy ? ry[l] : cx<T>{T(0), T(0)};
    }
#pragma unroll
    for (int r = 0; r < kPerT; ++r) {
        const int t = tid + r * kInvThreads;
        if (t < my) st[t] = vt[r];
    }
#pragma unroll
    for (int r = 0; r < kPerL; ++r) {
        const int l = tid + r * kInvThreads;
        if (l <= hy) {
            const cx<T> X = vx[r], Y = vy[r];
            // conjugated inputs for conj(FFT(conj(.)))
            a[sw(l)] = conj(X + mul_pos_i(Y));
            if (l > 0 && l < hy) a[sw(my - l)] = conj(conj(X) + mul_pos_i(conj(Y)));
        }
    }
    // the potential's row (with bp) is staged beside the field's
    cx<T> *a2 = b + my;
    cx<T> *b2 = a2 + my;
    if (bp) {
        const cx<T> *rp = bp + (size_t)(i + 1) * (hy + 1);
        for (int l = tid; l <= hy; l += kInvThreads) {
            const cx<T> P = rp[l];
            a2[sw(l)] = conj(P);
            if (l > 0 && l < hy) a2[sw(my - l)] = P;
        }
    }
    __syncthreads();
    // wave 0 transforms and stores the field row, wave 1 the potential's
    const int wave = tid >> 6, lane = tid & 63;
    const bool field_row = i >= 0 && i < nx;
    if (wave == 0 && field_row) {
        const cx<T> *r = fft_wave(a, b, my, log2my, st, lane);
        if (ef) {
            for (int j = lane; j < ny; j += 64) ef[(size_t)i * ny + j] = conj(r[sw(j)]);
        } else {
            for (int j = lane; j < ny; j += 64) {
                const cx<T> z = conj(r[sw(j)]);
                ex[(size_t)i * ny + j] = z.re;
                ey[(size_t)i * ny + j] = z.im;
            }
        }
    }
    if (wave == 1 && bp) {
        const cx<T> *r2 = fft_wave(a2, b2, my, log2my, st, lane);
        T *row = phi + (size_t)(i + 1) * (ny + 2);
        for (int j = lane - 1; j <= ny; j += 64) row[j + 1] = r2[sw(j < 0 ? my - 1 : j)].re;
    }
}

template <typename T>
__global__ void __launch_bounds__(kInvThreads)
    k_rows_inv(const cx<T> *__restrict__ bx, const cx<T> *__restrict__ by, int nx, int ny, int my,
               int log2my, const cx<T> *__restrict__ tw, T *__restrict__ ex, T *__restrict__ ey,
               cx<T> *__restrict__ ef, const cx<T> *__restrict__ bp, T *__restrict__ phi)
{
    // workgroups nx and nx + 1 (launched with the potential) take rows -1 and nx
    const int r = (int)blockIdx.x;
    const int i = r < nx ? r : (r == nx ? -1 : nx);
    rows_inv_body<T>(bx, by, nx, ny, my, log2my, tw, ex, ey, ef, i, bp, phi);
}

template <typename T>
__global__ void __launch_bounds__(kInvThreads) k_rows_inv_batched(BatchLaunch b)
{
    const BatchInstance &I = b.inst[b.row_inst[blockIdx.x]];
    rows_inv_body<T>((const cx<T> *)I.spec_bx, (const cx<T> *)I.spec_by, I.nx, I.ny, I.my,
                     I.log2_my, (const cx<T> *)I.stw_y + I.my + 1, nullptr, nullptr, (cx<T> *)I.ef,
                     (int)blockIdx.x - I.row_block0);
}

template <typename T>
hipError_t launch_tail(hipStream_t s, const SolveWorkspace &w, void *ex, void *ey, void *ef)
{
    const bool want_phi = w.want_phi;
    const size_t col_lds = 5 * sizeof(cx<T>) * (size_t)w.mx;
    const size_t inv_lds = (want_phi ? 5 : 3) * sizeof(cx<T>) * (size_t)w.my;
    cx<T> *bp = want_phi ? (cx<T> *)w.spec_p : nullptr;
    hipLaunchKernelGGL(k_cols<T>, dim3(w.my / 2 + 1), dim3(kColThreads), col_lds, s,
                       (const cx<T> *)w.spec_a, w.nx, w.my / 2, w.mx, w.log2_mx, (const cx<T> *)w.stw_x,
                       (const T *)w.ghat_t, (const T *)w.sx, (const T *)w.sy, (cx<T> *)w.spec_bx,
                       (cx<T> *)w.spec_by, w.pipe, bp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rows_inv<T>, dim3(w.nx + (want_phi ? 2 : 0)), dim3(kInvThreads), inv_lds, s,
                       (const cx<T> *)w.spec_bx, (const cx<T> *)w.spec_by, w.nx, w.ny, w.my,
                       w.log2_my, (const cx<T> *)w.stw_y + w.my + 1, (T *)ex, (T *)ey, (cx<T> *)ef,
                       (const cx<T> *)bp, want_phi ? (T *)w.phi : (T *)nullptr);
    return hipGetLastError();
}

template <typename T, bool FROM_PARTIALS>
hipError_t launch_solve_t(hipStream_t s, const SolveWorkspace &w, const DepositTarget &dep,
                          int nblocks, const int64_t *q, double scale, void *ex, void *ey,
                          void *ef)
{
    // the line tables come from the partials of a depositing pass only
    LineSpec line = FROM_PARTIALS ? w.line : LineSpec{};
    size_t row_lds = rows_fwd_hdr_offset<T>(w.ny, w.my) +
                     (FROM_PARTIALS ? sizeof(BlockHeader) * (size_t)std::max(nblocks, 1) : 0);
    if (line.nz > 0) row_lds = std::max(row_lds, sizeof(unsigned long long) * (size_t)kRowThreads);
    hipLaunchKernelGGL((k_rows_fwd<T, FROM_PARTIALS>), dim3(w.nx + (line.nz > 0 ? 1 : 0)),
                       dim3(kRowThreads), row_lds, s, dep, nblocks, q, scale, w.nx, w.ny, w.my,
                       w.log2_my, (const cx<T> *)w.stw_y, (cx<T> *)w.spec_a, w.pipe, line);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_tail<T>(s, w, ex, ey, ef);
}

template <typename T>
hipError_t launch_solve_batched_t(hipStream_t s, const BatchLaunch &b, int rows, int cols,
                                  int max_mx, int max_ny, int max_my, int max_pass_blocks)
{
    const int mmx = max_mx, mmy = max_my;
    const size_t row_lds = rows_fwd_hdr_offset<T>(max_ny, mmy) +
                           sizeof(BlockHeader) * (size_t)std::max(max_pass_blocks, 1);
    const size_t col_lds = 5 * sizeof(cx<T>) * (size_t)mmx;
    const size_t inv_lds = 3 * sizeof(cx<T>) * (size_t)mmy;
    if (max_ny <= 128 && mmy / 2 <= 128)
        hipLaunchKernelGGL((k_rows_fwd_batched<T, 128>), dim3(rows), dim3(128), row_lds, s, b);
    else
        hipLaunchKernelGGL((k_rows_fwd_batched<T, 256>), dim3(rows), dim3(256), row_lds, s, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cols_batched<T>, dim3(cols), dim3(kColThreads), col_lds, s, b);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rows_inv_batched<T>, dim3(rows), dim3(kInvThreads), inv_lds, s, b);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_solve_batched(hipStream_t s, const BatchLaunch &b, bool mixed, int rows,
                                int cols, int max_mx, int max_ny, int max_my, int max_pass_blocks)
{
    return mixed ? launch_solve_batched_t<float>(s, b, rows, cols, max_mx, max_ny, max_my,
                                                 max_pass_blocks)
                 : launch_solve_batched_t<double>(s, b, rows, cols, max_mx, max_ny, max_my,
                                                  max_pass_blocks);
}

hipError_t launch_reduce(hipStream_t s, const DepositTarget &dep, int blocks_used, int nx, int ny,
                         int64_t *q, int64_t *n_in)
{
    hipLaunchKernelGGL(k_reduce, dim3(nx), dim3(kRowThreads), 0, s, dep, blocks_used, nx, ny, q,
                       n_in);
    return hipGetLastError();
}

hipError_t launch_solve(hipStream_t s, const SolveWorkspace &w, const int64_t *q, double scale,
                        void *ex, void *ey, void *ef)
{
    DepositTarget none{};
    return w.mixed ? launch_solve_t<float, false>(s, w, none, 0, q, scale, ex, ey, ef)
                   : launch_solve_t<double, false>(s, w, none, 0, q, scale, ex, ey, ef);
}

hipError_t launch_solve_partials(hipStream_t s, const SolveWorkspace &w, const DepositTarget &dep,
                                 int blocks_used, double scale, void *ef)
{
    return w.mixed ? launch_solve_t<float, true>(s, w, dep, blocks_used, nullptr, scale, nullptr,
                                                 nullptr, ef)
                   : launch_solve_t<double, true>(s, w, dep, blocks_used, nullptr, scale, nullptr,
                                                  nullptr, ef);
}

}  // namespace scpic
