// Grid-side kernels of libscpic for gfx950: the open-boundary Poisson solve
// as a zero-padded (2nx x 2ny) FFT convolution with the free-space Green's
// function (Hockney's method), with the centred-difference field taken in the
// spectrum.  Hand-written radix-4/2 Stockham FFTs in LDS, one wavefront per
// transform; no vendor FFT library.
//
// Data flow for a charge grid q (nx x ny int64, rows i along x):
//   k_rows_fwd   rows i, i+1 packed as one complex sequence of length my
//                (zero-padded), FFT along y, untangled into the two real-input
//                half spectra l = 0..ny                     -> A^T [ny+1][nx]
//   k_cols       per column l: FFT along x (length mx, zero-padded), multiply
//                by the real Green's spectrum G^(k,l) (normalisation folded
//                in), then two inverse FFTs: one of -i sin(2 pi k/mx)/dx * Phi
//                (the x central difference) and one of Phi, scaled by
//                -i sin(2 pi l/my)/dy (the y central difference); rows
//                0..nx-1 kept                                -> Bx, By [nx][ny+1]
//   k_rows_inv   per row i: both half spectra packed as Ex + i Ey, completed
//                by Hermitian symmetry, one inverse FFT     -> ex, ey [nx][ny]
// Taking the differences in the spectrum keeps the large constant part of
// the potential out of the field's rounding, which matters for the FP32 form.
#include "scpic_internal.h"

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
// -i * a
template <typename T>
__device__ __forceinline__ cx<T> mul_neg_i(cx<T> a) { return {a.im, -a.re}; }
// +i * a
template <typename T>
__device__ __forceinline__ cx<T> mul_pos_i(cx<T> a) { return {-a.im, a.re}; }

// Forward DFT X[k] = sum_n x[n] exp(-2 pi i n k / L) of the sequence in LDS
// buffer a (length L = 2^log2L), computed by the nthr threads of the
// workgroup (all of which must call this), ping-ponging with buffer b.
// Stockham autosort: one radix-2 stage first when log2L is odd, then radix-4
// stages; each stage reads sub-transform inputs a stride L/r apart, applies
// the twiddles exp(-2 pi i m k / (Ns r)) and writes the r outputs Ns apart.
// tw[t] = exp(-2 pi i t / L).  Returns the buffer holding X in natural order.
template <typename T>
__device__ cx<T> *fft_lds(cx<T> *a, cx<T> *b, int L, int log2L, const cx<T> *__restrict__ tw,
                          int tid, int nthr)
{
    __syncthreads();
    int ns = 1;
    if (log2L & 1) {
        const int h = L >> 1;
        for (int j = tid; j < h; j += nthr) {
            const cx<T> u = a[j], v = a[j + h];
            b[2 * j] = u + v;
            b[2 * j + 1] = u - v;
        }
        cx<T> *t = a;
        a = b;
        b = t;
        ns = 2;
        __syncthreads();
    }
    const int q = L >> 2;
    while (ns < L) {
        for (int j = tid; j < q; j += nthr) {
            const int k = j & (ns - 1);
            const int step = (L / (4 * ns)) * k;
            const cx<T> a0 = a[j];
            const cx<T> a1 = cmul(a[j + q], tw[step]);
            const cx<T> a2 = cmul(a[j + 2 * q], tw[2 * step]);
            const cx<T> a3 = cmul(a[j + 3 * q], tw[3 * step]);
            const cx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = a1 - a3;
            const int base = (j - k) * 4 + k;
            b[base] = t0 + t2;
            b[base + ns] = t1 + mul_neg_i(t3);
            b[base + 2 * ns] = t0 - t2;
            b[base + 3 * ns] = t1 + mul_pos_i(t3);
        }
        cx<T> *t = a;
        a = b;
        b = t;
        ns *= 4;
        __syncthreads();
    }
    return a;
}

constexpr int kFftThreads = 64;

// Rows 2r and 2r+1 of rho = q * scale, zero-padded to my, as one complex FFT
// along y; the two real-input spectra are separated with
//   A0[l] = (Z[l] + conj Z[my-l]) / 2,   A1[l] = -i (Z[l] - conj Z[my-l]) / 2.
template <typename T>
__global__ void __launch_bounds__(kFftThreads)
    k_rows_fwd(const int64_t *__restrict__ q, double scale, int nx, int ny, int my, int log2my,
               const cx<T> *__restrict__ tw, cx<T> *__restrict__ at)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T> *twl = reinterpret_cast<cx<T> *>(smem_raw);
    cx<T> *a = twl + my;
    cx<T> *b = a + my;
    const int tid = threadIdx.x;
    for (int t = tid; t < my; t += kFftThreads) twl[t] = tw[t];
    const int i0 = 2 * blockIdx.x;
    const int64_t *r0 = q + (size_t)i0 * ny;
    const int64_t *r1 = r0 + ny;
    for (int j = tid; j < my; j += kFftThreads) {
        cx<T> z = {T(0), T(0)};
        if (j < ny) {
            z.re = (T)((double)r0[j] * scale);
            z.im = (T)((double)r1[j] * scale);
        }
        a[j] = z;
    }
    const cx<T> *r = fft_lds(a, b, my, log2my, twl, tid, kFftThreads);
    for (int l = tid; l <= ny; l += kFftThreads) {
        const cx<T> zl = r[l];
        const cx<T> zm = conj(r[(my - l) & (my - 1)]);
        const cx<T> s = zl + zm, d = zl - zm;
        at[(size_t)l * nx + i0] = {s.re * T(0.5), s.im * T(0.5)};
        at[(size_t)l * nx + i0 + 1] = mul_neg_i(cx<T>{d.re * T(0.5), d.im * T(0.5)});
    }
}

// Column l of the row spectra: forward FFT along x, times the Green's
// spectrum, and the two differentiated inverse transforms.
template <typename T>
__global__ void __launch_bounds__(kFftThreads)
    k_cols(const cx<T> *__restrict__ at, int nx, int ny, int mx, int log2mx,
           const cx<T> *__restrict__ tw, const T *__restrict__ ghat_t, const T *__restrict__ sx,
           const T *__restrict__ sy, cx<T> *__restrict__ bx, cx<T> *__restrict__ by)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T> *twl = reinterpret_cast<cx<T> *>(smem_raw);
    cx<T> *a = twl + mx;
    cx<T> *b = a + mx;
    cx<T> *c = b + mx;
    T *gl = reinterpret_cast<T *>(c + mx);
    T *sxl = gl + mx;
    const int tid = threadIdx.x;
    const int l = blockIdx.x;
    const cx<T> *col = at + (size_t)l * nx;
    const T *g = ghat_t + (size_t)l * mx;
    // stage every input of the column in LDS up front (one round of loads)
    for (int i = tid; i < mx; i += kFftThreads) {
        twl[i] = tw[i];
        gl[i] = g[i];
        sxl[i] = sx[i];
        a[i] = i < nx ? col[i] : cx<T>{T(0), T(0)};
    }
    const T syl = sy[l];
    cx<T> *r = fft_lds(a, b, mx, log2mx, twl, tid, kFftThreads);
    // Inverse transforms as conj(FFT(conj(.))): stage the conjugated inputs.
    for (int k = tid; k < mx; k += kFftThreads) {
        const T gk = gl[k];
        const cx<T> phi = {r[k].re * gk, r[k].im * gk};
        c[k] = conj(phi);
        const cx<T> dx = mul_neg_i(cx<T>{phi.re * sxl[k], phi.im * sxl[k]});
        r[k] = conj(dx);
    }
    cx<T> *o = (r == a) ? b : a;
    const cx<T> *rx = fft_lds(r, o, mx, log2mx, twl, tid, kFftThreads);
    for (int i = tid; i < nx; i += kFftThreads) bx[(size_t)i * (ny + 1) + l] = conj(rx[i]);
    // rx may alias r or o; c is untouched.  Use the two free buffers for the
    // second inverse transform.
    cx<T> *f0 = c;
    cx<T> *f1 = (rx == a) ? b : a;
    const cx<T> *ry = fft_lds(f0, f1, mx, log2mx, twl, tid, kFftThreads);
    for (int i = tid; i < nx; i += kFftThreads) {
        const cx<T> p = conj(ry[i]);
        by[(size_t)i * (ny + 1) + l] = mul_neg_i(cx<T>{p.re * syl, p.im * syl});
    }
}

// Row i: Z[l] = Bx[l] + i By[l] for l = 0..ny and Z[my-l] = conj(Bx[l]) +
// i conj(By[l]) for 0 < l < ny; one inverse FFT gives ex + i ey.  Written
// either as two arrays (ex, ey) or interleaved into ef (Ex, Ey per node).
template <typename T>
__global__ void __launch_bounds__(kFftThreads)
    k_rows_inv(const cx<T> *__restrict__ bx, const cx<T> *__restrict__ by, int nx, int ny, int my,
               int log2my, const cx<T> *__restrict__ tw, T *__restrict__ ex, T *__restrict__ ey,
               cx<T> *__restrict__ ef)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T> *twl = reinterpret_cast<cx<T> *>(smem_raw);
    cx<T> *a = twl + my;
    cx<T> *b = a + my;
    const int tid = threadIdx.x;
    const int i = blockIdx.x;
    for (int t = tid; t < my; t += kFftThreads) twl[t] = tw[t];
    const cx<T> *rx = bx + (size_t)i * (ny + 1);
    const cx<T> *ry = by + (size_t)i * (ny + 1);
    for (int l = tid; l <= ny; l += kFftThreads) {
        const cx<T> X = rx[l], Y = ry[l];
        // conjugated inputs for conj(FFT(conj(.)))
        a[l] = conj(X + mul_pos_i(Y));
        if (l > 0 && l < ny) a[my - l] = conj(conj(X) + mul_pos_i(conj(Y)));
    }
    const cx<T> *r = fft_lds(a, b, my, log2my, twl, tid, kFftThreads);
    if (ef) {
        for (int j = tid; j < ny; j += kFftThreads) ef[(size_t)i * ny + j] = conj(r[j]);
    } else {
        for (int j = tid; j < ny; j += kFftThreads) {
            const cx<T> z = conj(r[j]);
            ex[(size_t)i * ny + j] = z.re;
            ey[(size_t)i * ny + j] = z.im;
        }
    }
}

template <typename T>
hipError_t launch_solve_t(hipStream_t s, const SolveWorkspace &w, const int64_t *q, double scale,
                          void *ex, void *ey, void *ef)
{
    const size_t row_lds = 3 * sizeof(cx<T>) * (size_t)w.my;
    const size_t col_lds = (4 * sizeof(cx<T>) + 2 * sizeof(T)) * (size_t)w.mx;
    hipLaunchKernelGGL(k_rows_fwd<T>, dim3(w.nx / 2), dim3(kFftThreads), row_lds, s, q, scale,
                       w.nx, w.ny, w.my, w.log2_my, (const cx<T> *)w.tw_y, (cx<T> *)w.spec_a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cols<T>, dim3(w.ny + 1), dim3(kFftThreads), col_lds, s,
                       (const cx<T> *)w.spec_a, w.nx, w.ny, w.mx, w.log2_mx, (const cx<T> *)w.tw_x,
                       (const T *)w.ghat_t, (const T *)w.sx, (const T *)w.sy, (cx<T> *)w.spec_bx,
                       (cx<T> *)w.spec_by);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rows_inv<T>, dim3(w.nx), dim3(kFftThreads), row_lds, s,
                       (const cx<T> *)w.spec_bx, (const cx<T> *)w.spec_by, w.nx, w.ny, w.my,
                       w.log2_my, (const cx<T> *)w.tw_y, (T *)ex, (T *)ey, (cx<T> *)ef);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_solve(hipStream_t s, const SolveWorkspace &w, const int64_t *q, double scale,
                        void *ex, void *ey, void *ef)
{
    return w.mixed ? launch_solve_t<float>(s, w, q, scale, ex, ey, ef)
                   : launch_solve_t<double>(s, w, q, scale, ex, ey, ef);
}

}  // namespace scpic
