// Internal declarations shared by the host-side translation units of libscpic.
// Not installed; the public interface is include/scpic.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "scpic.h"

namespace scpic {

// Fixed-point charge: 12 fractional bits per axis, 2^24 units per particle.
constexpr int kFracBits = 12;
constexpr int kFracOne = 1 << kFracBits;  // 4096
constexpr double kChargeOne = 16777216.0;  // 2^24

// Elements a single particle pass can carry in its kernel arguments.
constexpr int kMaxPassElements = 12;
// Static LDS a six-dimensional pass may declare (its box and count words and
// its copy of the element parameters); its dynamic LDS budget is the
// device's per-workgroup LDS minus this (256 bytes for the four-dimensional
// passes).
constexpr int kPassStaticLds = 2048;

// Most split steps a thick sextupole may take.
constexpr int kMaxSextSteps = 1024;

// Largest FFT length (the padded length of the largest grid side, 256) and
// largest grid.
constexpr int kMaxFft = 512;
constexpr int kMaxCells = 65536;

// Most workgroups a depositing pass may use (one partial grid each).
constexpr int kMaxPassBlocks = 512;

// Per-block header written by a depositing pass: bounding box of the cells it
// touched (inclusive; empty when i0 > i1) and how many particles it deposited.
struct BlockHeader {
    int32_t i0, i1, j0, j1;
    int32_t count;
    int32_t pad[3];
};

// Grid geometry as the kernels see it.  inv_dx / inv_dy are 1.0/dx and
// 1.0/dy computed once on the host in FP64.
struct GridGeom {
    int32_t nx, ny;
    double x_min, y_min, inv_dx, inv_dy;
};

// Elements of one pass, passed by value in the kernel arguments (read with
// scalar loads, uniform across the wave).  A thick quadrupole's p[3..8] hold
// values derived on the host from k1 and L: phi0 = sqrt|k1| L, sin, cos,
// sinh and cosh of phi0, and 1/sqrt|k1| (0 when k1 = 0).
struct PassElements {
    int32_t n_el;
    int32_t kind[kMaxPassElements];
    double p[kMaxPassElements][16];
};

// Device-side buffers of the charge partials.  Workgroup b of a depositing
// pass writes the cells (i, j) of its bounding box to
// partial[(i * max_blocks + b) * ny + j]: the partials of one grid row are
// contiguous, so the row that reduces them reads one contiguous span.
struct DepositTarget {
    uint32_t *partial;            // [nx][max_blocks][ny]
    BlockHeader *header;          // [max_blocks]
    unsigned long long *carry;    // [nx*ny] whole 2^32 overflows of LDS cells
    int32_t max_blocks;
};

struct ParticlePtrs {
    double *x, *px, *y, *py;
    double *sigma;         // longitudinal pair, may be null (four-dimensional)
    double *psigma;
    const float *w;  // per-particle kick weight (2.5D line density), may be null
    uint8_t *lost;
    int64_t n;
    // The arrays are far larger than the last-level cache: the pass streams
    // the four transverse coordinates with non-temporal loads and stores.
    bool stream;
};

// Particle arrays above this many bytes are streamed (half the MI355X's
// 256 MB last-level cache; below it the arrays stay cached between passes).
constexpr int64_t kStreamBytes = 128ll << 20;

// Line density of a long bunch (Sec. IV) as a pass sees it: the line of nz
// nodes z_min + k dz, the node tables of the last solve (lambda/lambda_peak
// and lambda'/lambda_peak) and its node potential for the kick, and the
// per-workgroup histograms [max_blocks][nz] a depositing pass writes.
struct LineSpec {
    int32_t nz;
    double z_min, inv_dz, dz, gamma0;
    double *lw, *ld;                 // [nz], written by the grid phase
    const void *phi;                 // [(nx+2)*(ny+2)] node potential (nodes -1..n)
    unsigned long long *partial;     // [max_blocks][nz]
};

// Twiddles of the radix-4 stages of an L-point FFT (L = 2^log2L) as the
// grid kernels' one-wave Stockham FFT reads them, stage by stage, so that the
// lanes of a wave read them at consecutive addresses (or all at one): the
// stage that combines sub-transforms of length ns (ns = 1, 4, 16, ..., or
// 2, 8, 32, ... after the radix-2 stage of an odd log2L) keeps W^(m span k),
// W = exp(-2 pi i / L), span = L / (4 ns), for k < ns and m = 1, 2, 3 at entry
// ns - c + 3 k + m - 1, where c = 1 for even log2L and 2 for odd: L - c
// entries in all.  stage_twiddle_exponent gives the exponent m span k of
// entry e.
__host__ __device__ constexpr int stage_twiddle_count(int L, int log2L)
{
    return L - ((log2L & 1) ? 2 : 1);
}
inline int stage_twiddle_exponent(int e, int L, int log2L)
{
    const int c = (log2L & 1) ? 2 : 1;
    int ns = c;
    while (4 * ns - c <= e) ns *= 4;
    const int r = e - (ns - c);
    const int k = r / 3, m = r - 3 * k + 1;
    return m * (L / (4 * ns)) * k;
}

// Most nodes of a line-density grid.
constexpr int kMaxLineNodes = 512;

// One beam of a batch, as the batched kernels see it: its particles (a
// contiguous range of the concatenated arrays), its grid, its partials and
// its solve workspace, and where its workgroups start in each batched launch.
struct BatchInstance {
    int64_t p0, n;                     // particles [p0, p0 + n)
    int32_t pass_block0, pass_blocks;  // its workgroups in a batched pass
    int32_t row_block0, col_block0;    // its first workgroup in the row / column kernels
    GridGeom g;
    DepositTarget dep;                 // max_blocks == pass_blocks
    int32_t nx, ny, mx, my, log2_mx, log2_my;
    double scale;                      // 1 / (2^24 N0): charge units -> rho
    const void *stw_x, *stw_y, *ghat_t, *sx, *sy;  // twiddle tables as in SolveWorkspace
    void *spec_a, *spec_bx, *spec_by;
    void *ef;                          // interleaved node field
};

// What one batched pass applies to one beam: its pending kick strength and
// the elements up to its next space-charge location.
struct BatchStep {
    double kappa;
    PassElements els;
};

// Device tables of a batch: the beams and, per batched launch, the beam of
// each workgroup.
struct BatchLaunch {
    const BatchInstance *inst;
    const uint16_t *pass_inst;  // [total pass workgroups]
    const uint16_t *row_inst;   // [sum nx]: row-forward and row-inverse kernels
    const uint16_t *col_inst;   // [sum (my/2 + 1)]: column kernel
    int32_t n_inst;
};

// ---- launchers (particles.hip) ------------------------------------------
// ef: interleaved node field (Ex, Ey per node), double or float per mixed.
// line: the long-bunch line density (kick scaled by lambda/lambda_peak, the
// longitudinal kick, the line histogram with the deposit), or null.
// bspline_phi: the node potential (nodes -1..nx by -1..ny) when the kick takes
// the B-spline field (Sec. IV-C) instead of gathering ef; not with a line.
hipError_t launch_pass(hipStream_t s, const ParticlePtrs &p, const GridGeom &g, bool kick,
                       bool mixed, const void *ef, double kappa, const PassElements &els,
                       bool deposit, const DepositTarget &dep, int blocks, int threads,
                       const LineSpec *line = nullptr, const void *bspline_phi = nullptr);

// Beam moments for scpic_diagnose: sums[0..5] = alive count and the sums of
// x, px, y, py over the alive particles; sums[6..11] = the sums of the
// centred products dx^2, dpx^2, dx dpx, dy^2, dpy^2, dy dpy.  part: scratch of
// kMomentBlocks * kMoments doubles.
constexpr int kMomentBlocks = 256;
constexpr int kMoments = 6;
hipError_t launch_moments(hipStream_t s, const ParticlePtrs &p, double *part, double *sums);

// Copy (ex, ey) into the interleaved field ef, or back.
hipError_t launch_interleave(hipStream_t s, bool mixed, bool to_interleaved, void *ex, void *ey,
                             void *ef, int ncell);

hipError_t prepare_pass_kernels(size_t lds_per_workgroup);

// True when els holds a thick element (the pass then needs sigma, p_sigma).
bool has_thick(const PassElements &els);

// One particle pass over every beam of a batch (blocks = total pass
// workgroups of the batch); steps[beam] holds each beam's kick and elements;
// six when any beam's elements in this pass are thick.
hipError_t launch_pass_batched(hipStream_t s, const BatchLaunch &b, const ParticlePtrs &all,
                               const BatchStep *steps, bool kick, bool mixed, bool deposit,
                               bool six, int blocks, int threads);

// Exact charge grid q (int64) and deposited count from the partials of the
// last depositing pass (blocks_used workgroups); clears the carry grid.
hipError_t launch_reduce(hipStream_t s, const DepositTarget &dep, int blocks_used, int nx, int ny,
                         int64_t *q, int64_t *n_in);

// ---- launchers (fft_solve.hip) -------------------------------------------
struct SolveWorkspace {
    int nx, ny, mx, my, log2_mx, log2_my;  // mx, my: FFT lengths, powers of two >= 2n
    bool mixed;
    bool pipe;           // grounded rectangular pipe instead of the open boundary
    // complex twiddle tables: stw_x the stage twiddles of the mx-point FFT
    // [mx]; stw_y the plain exp(-2 pi i l / my) for l = 0..hy, then the stage
    // twiddles of the hy-point FFT at hy + 1 and of the my-point FFT at my + 1
    // [2 my + 1]
    void *stw_x, *stw_y;
    void *ghat_t;        // [my/2+1][mx] real Green's spectrum / (mx my), transposed
    void *sx, *sy;       // [mx] sin(2 pi k / mx)/dx, [my/2+1] sin(2 pi l / my)/dy
    void *spec_a;        // [my/2+1][nx] complex, rows transformed
    void *spec_bx, *spec_by;  // [nx][my/2+1] complex, after the column pass
    // node potential (want_phi; for the line density or the B-spline gather):
    // the potential's column-inverse spectrum [nx+2][my/2+1] complex (rows
    // -1..nx) and the potential on nodes -1..nx by -1..ny [(nx+2)*(ny+2)];
    // with line.nz > 0 the line tables reduced from the pass's histograms
    bool want_phi = false;
    void *spec_p = nullptr;
    void *phi = nullptr;
    LineSpec line{};
};

// Field of charge grid q: to separate arrays ex, ey (ef == nullptr) or
// interleaved into ef.
hipError_t launch_solve(hipStream_t s, const SolveWorkspace &w, const int64_t *q, double scale,
                        void *ex, void *ey, void *ef);

// Field straight from the partials of the last depositing pass (the exact
// integer reduction is fused into the first FFT stage), interleaved into ef.
hipError_t launch_solve_partials(hipStream_t s, const SolveWorkspace &w, const DepositTarget &dep,
                                 int blocks_used, double scale, void *ef);

// Field of every beam of a batch from the partials of its last batched pass,
// interleaved into each beam's ef: rows = sum of nx, cols = sum of (my/2 + 1);
// max_mx, max_ny, max_my bound every beam's (padded) lengths and
// max_pass_blocks every beam's pass workgroups.
hipError_t launch_solve_batched(hipStream_t s, const BatchLaunch &b, bool mixed, int rows,
                                int cols, int max_mx, int max_ny, int max_my, int max_pass_blocks);

// Green's spectrum helper on the host (api.hip): fills ghat_t (FP64,
// [my/2+1][mx]) for the mx x my periodic kernel (mx >= 2 nx, my >= 2 ny).
void green_spectrum_host(int mx, int my, double dx, double dy, double *ghat_t);

// The grounded pipe's counterpart of ghat_t (same layout and normalisation):
// the inverse of the 5-point Laplacian's eigenvalue per mode of the odd
// extension, times -2 pi / (dx dy), mode (0, 0) zero.
void pipe_spectrum_host(int nx, int ny, double dx, double dy, double *ghat_t);

}  // namespace scpic
