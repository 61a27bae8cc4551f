// Host side of libscpic: the C ABI declared in include/scpic.h.  Contexts own
// every workspace (allocated once in scpic_create); calls validate their
// arguments, then enqueue kernels on the context's stream.  scpic_track turns
// the one-turn element sequence into a schedule of fused particle passes and
// grid solves and replays it as a captured HIP graph per turn.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "scpic_internal.h"

using namespace scpic;

namespace {

thread_local std::string g_last_error;

scpic_status fail(scpic_status code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

scpic_status fail_hip(hipError_t e, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return SCPIC_EHIP;
}

#define SCPIC_HIP_TRY(expr, what)                  \
    do {                                           \
        hipError_t e_ = (expr);                    \
        if (e_ != hipSuccess) return fail_hip(e_, what); \
    } while (0)

int ilog2(int v)
{
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// FFT length of an axis of n nodes: the smallest power of two >= 2 n.  The
// open-boundary kernel sampled at min(k, m - k) then makes the cyclic
// convolution equal the linear one on nodes -1..n for any such m.
int fft_len(int n) { return 1 << ilog2(2 * n); }

// One launch of the particle pass, as scheduled by scpic_track.
struct PassOp {
    bool kick;
    double kappa;
    PassElements els;
    bool deposit;
};

struct GraphEntry {
    std::vector<unsigned char> key;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
};

}  // namespace

struct scpic_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    scpic_grid grid{};
    GridGeom geom{};
    bool mixed = false;
    int n_cu = 0;
    int max_blocks = 0;
    int pass_blocks = 0;  // 0 = automatic
    int pass_threads = 1024;
    bool use_graph = true;
    int last_deposit_blocks = 0;

    DepositTarget dep{};
    SolveWorkspace sw{};
    void *ef = nullptr;  // internal field, interleaved (Ex, Ey) per node

    // long-bunch line density (scpic_set_line_density); line.nz = 0: off
    LineSpec line{};
    std::vector<void *> line_mem;
    // kick field from the B-spline surface of the potential (SCPIC_OPT_GATHER)
    bool bspline = false;
    // scpic_diagnose: per-workgroup moment sums and the two passes' totals
    double *diag_part = nullptr;
    double *diag_sums = nullptr;

    std::vector<void *> allocations;
    std::vector<GraphEntry> graphs;
    uint64_t use_counter = 0;
};

namespace {

size_t field_elem_size(const scpic_ctx *c) { return c->mixed ? sizeof(float) : sizeof(double); }

scpic_status dev_alloc(scpic_ctx *c, void **p, size_t bytes)
{
    hipError_t e = hipMalloc(p, bytes ? bytes : 1);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(SCPIC_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    c->allocations.push_back(*p);
    return SCPIC_OK;
}

void free_line(scpic_ctx *c)
{
    for (void *p : c->line_mem) hipFree(p);
    c->line_mem.clear();
    c->line = LineSpec{};
    c->sw.line = LineSpec{};
    c->sw.want_phi = c->bspline;
}

// The node potential (nodes -1..nx by -1..ny) and its spectrum, allocated
// once, when the line density or the B-spline field first needs them.
scpic_status ensure_potential(scpic_ctx *c)
{
    if (c->sw.phi) return SCPIC_OK;
    const size_t es = field_elem_size(c);
    void *phi = nullptr, *spec = nullptr;
    if (scpic_status st = dev_alloc(c, &phi, es * (size_t)(c->grid.nx + 2) * (c->grid.ny + 2)))
        return st;
    if (scpic_status st = dev_alloc(c, &spec, 2 * es * (size_t)(c->grid.nx + 2) * (c->sw.my / 2 + 1)))
        return st;
    SCPIC_HIP_TRY(hipMemset(phi, 0, es * (size_t)(c->grid.nx + 2) * (c->grid.ny + 2)), "hipMemset");
    c->sw.phi = phi;
    c->sw.spec_p = spec;
    return SCPIC_OK;
}

void drop_graphs(scpic_ctx *c)
{
    for (auto &g : c->graphs)
        if (g.exec) hipGraphExecDestroy(g.exec);
    c->graphs.clear();
}

void free_all(scpic_ctx *c)
{
    free_line(c);
    for (auto &g : c->graphs)
        if (g.exec) hipGraphExecDestroy(g.exec);
    c->graphs.clear();
    for (void *p : c->allocations) hipFree(p);
    c->allocations.clear();
    if (c->capture_stream) hipStreamDestroy(c->capture_stream);
    c->capture_stream = nullptr;
}

scpic_status check_ctx(const scpic_ctx *c)
{
    if (!c) return fail(SCPIC_EINVAL, "ctx is NULL");
    return SCPIC_OK;
}

scpic_status check_grid(const scpic_grid *grid)
{
    if (!(grid->dx > 0.0) || !(grid->dy > 0.0) || !std::isfinite(grid->dx) ||
        !std::isfinite(grid->dy) || !std::isfinite(grid->x_min) || !std::isfinite(grid->y_min))
        return fail(SCPIC_EINVAL, "grid spacing must be positive and finite, origin finite");
    if (grid->nx < 8 || grid->nx > 256 || grid->ny < 8 || grid->ny > 256 || grid->ny % 4 != 0)
        return fail(SCPIC_EUNSUPPORTED, "nx must be in [8, 256] and ny a multiple of 4 in [8, 256]");
    if ((int64_t)grid->nx * grid->ny > kMaxCells)
        return fail(SCPIC_EUNSUPPORTED, "nx * ny must not exceed 65536");
    return SCPIC_OK;
}

scpic_status check_parts(const scpic_particles *p)
{
    if (!p) return fail(SCPIC_EINVAL, "particles is NULL");
    if (p->n < 0) return fail(SCPIC_EINVAL, "particle count is negative");
    if (p->n > 0 && (!p->x || !p->px || !p->y || !p->py))
        return fail(SCPIC_EINVAL, "a particle coordinate pointer is NULL");
    return SCPIC_OK;
}

ParticlePtrs to_ptrs(const scpic_particles *p)
{
    ParticlePtrs r;
    r.x = p->x;
    r.px = p->px;
    r.y = p->y;
    r.py = p->py;
    r.sigma = p->sigma;
    r.psigma = p->psigma;
    r.w = p->w;
    r.lost = p->lost;
    r.n = p->n;
    const int64_t bytes_per = 8 * (4 + (p->sigma ? 1 : 0) + (p->psigma ? 1 : 0)) +
                              (p->w ? 4 : 0) + (p->lost ? 1 : 0);
    r.stream = p->n > kStreamBytes / bytes_per;
    return r;
}

// Workgroups of a pass over n particles.  A pass that kicks or deposits runs
// the depositing passes' count (one per compute unit unless set): workgroup b
// then owns the same particles as in the deposit that wrote header b, whose
// box sizes its tile and its staged field.  A pure push takes up to eight per
// compute unit.
int blocks_for(const scpic_ctx *c, int64_t n, bool lds_pass)
{
    if (n <= 0) return 0;
    const int64_t need = (n + c->pass_threads - 1) / c->pass_threads;
    const int64_t cap = lds_pass ? (c->pass_blocks > 0 ? c->pass_blocks : c->n_cu)
                                 : (int64_t)c->n_cu * 8;
    return (int)std::max<int64_t>(1, std::min<int64_t>(need, std::min<int64_t>(cap, c->max_blocks)));
}

// Non-SC elements of a host array, validated.
scpic_status collect_elements(const scpic_element *els, int32_t n_el,
                              std::vector<const scpic_element *> &out, bool allow_sc)
{
    if (n_el < 0) return fail(SCPIC_EINVAL, "element count is negative");
    if (n_el > 0 && !els) return fail(SCPIC_EINVAL, "elements pointer is NULL");
    for (int i = 0; i < n_el; ++i) {
        const int k = els[i].kind;
        const double *m = els[i].p;
        if (k != SCPIC_EL_LIN2X2 && k != SCPIC_EL_LIN4X4 && k != SCPIC_EL_SEXT_THIN &&
            k != SCPIC_EL_SC && k != SCPIC_EL_QUAD_THICK && k != SCPIC_EL_SEXT_THICK)
            return fail(SCPIC_EINVAL, "element " + std::to_string(i) + " has unknown kind " +
                                          std::to_string(k));
        if ((k == SCPIC_EL_QUAD_THICK || k == SCPIC_EL_SEXT_THICK) &&
            !(std::isfinite(m[0]) && std::isfinite(m[1]) && std::isfinite(m[2])))
            return fail(SCPIC_EINVAL, "element " + std::to_string(i) +
                                          ": thick element parameters must be finite");
        if (k == SCPIC_EL_SEXT_THICK &&
            !(m[3] >= 1.0 && m[3] <= (double)kMaxSextSteps && m[3] == std::floor(m[3])))
            return fail(SCPIC_EINVAL, "element " + std::to_string(i) +
                                          ": thick sextupole steps must be an integer in [1, " +
                                          std::to_string(kMaxSextSteps) + "]");
        if (k == SCPIC_EL_SC && !allow_sc) continue;
        out.push_back(&els[i]);
    }
    return SCPIC_OK;
}

// Thick elements advance sigma with p_sigma: the particles must carry both.
scpic_status check_longitudinal(const std::vector<const scpic_element *> &els,
                                const scpic_particles *p)
{
    if (p->n == 0 || (p->sigma && p->psigma)) return SCPIC_OK;
    for (const scpic_element *e : els)
        if (e->kind == SCPIC_EL_QUAD_THICK || e->kind == SCPIC_EL_SEXT_THICK)
            return fail(SCPIC_EINVAL, "thick elements need the particles' sigma and psigma");
    return SCPIC_OK;
}

// The elements [begin, end) of v as one pass's kernel arguments.  A thick
// quadrupole gets its on-momentum rotation computed here.  A drift (a thick
// sextupole without strength) next to a thick sextupole with the same
// 1/gamma0^2 is folded into that sextupole's first or last H0 flow, and
// adjacent drifts into one: the exact flows of H0 compose by adding their
// lengths, so this changes results only by rounding.  A thick sextupole's
// p[4] and p[5] carry the folded lead-in and tail lengths, p[6..9] its step
// lengths.
PassElements pack(const std::vector<const scpic_element *> &v, size_t begin, size_t end)
{
    PassElements pe;
    std::memset(&pe, 0, sizeof(pe));
    int k = 0;
    for (size_t i = begin; i < end; ++i) {
        const int kind = v[i]->kind;
        double m[16];
        std::memcpy(m, v[i]->p, sizeof(double) * 16);
        if (kind == SCPIC_EL_SEXT_THICK) {
            m[4] = 0.0;
            m[5] = 0.0;
            if (k > 0 && pe.kind[k - 1] == SCPIC_EL_SEXT_THICK && pe.p[k - 1][2] == m[2]) {
                double *q = pe.p[k - 1];
                const bool drift = m[0] == 0.0, prev_drift = q[0] == 0.0;
                if (drift && prev_drift) {
                    q[1] += m[1];
                    continue;
                }
                if (drift) {  // the tail of the previous sextupole
                    q[5] += m[1];
                    continue;
                }
                if (prev_drift) {  // the previous drift leads into this sextupole
                    const double lead = q[1];
                    std::memcpy(q, m, sizeof(double) * 16);
                    q[4] = lead;
                    continue;
                }
            }
        }
        if (kind == SCPIC_EL_QUAD_THICK) {
            // the on-momentum rotation of both planes, which the kernel
            // corrects per particle for its p_sigma
            const double w0 = std::sqrt(std::fabs(m[0])), phi0 = w0 * m[1];
            m[3] = phi0;
            m[4] = std::sin(phi0);
            m[5] = std::cos(phi0);
            m[6] = std::sinh(phi0);
            m[7] = std::cosh(phi0);
            m[8] = w0 > 0.0 ? 1.0 / w0 : 0.0;
            for (int j = 9; j < 16; ++j) m[j] = 0.0;
        }
        pe.kind[k] = kind;
        std::memcpy(pe.p[k], m, sizeof(double) * 16);
        ++k;
    }
    pe.n_el = k;
    // A thick sextupole's step lengths, the same for every particle, once
    // here (after the folding above, which changes p[1], p[4], p[5]) and with
    // the same operations the kernel would apply: p[6] = L / n and the
    // split's a h, c h and k2 h / 2 in p[7..9]; a drift's whole length in p[6].
    for (int e = 0; e < k; ++e) {
        if (pe.kind[e] != SCPIC_EL_SEXT_THICK) continue;
        double *q = pe.p[e];
        if (q[0] == 0.0) {
            q[6] = q[1] + q[4] + q[5];
        } else {
            constexpr double kC = 0.57735026918962576451;  // 1/sqrt(3)
            constexpr double kA = 0.5 * (1.0 - kC);
            const double h = q[1] / (double)(int)q[3];
            q[6] = h;
            q[7] = kA * h;
            q[8] = kC * h;
            q[9] = 0.5 * h * q[0];
        }
    }
    return pe;
}

// A run of non-SC elements between space-charge locations as one or more
// passes: the first carries the pending kick, the last the deposit.
void emit_segment(std::vector<PassOp> &ops, bool kick, double kappa,
                  const std::vector<const scpic_element *> &els, bool deposit)
{
    const size_t n = els.size();
    size_t at = 0;
    bool first = true;
    do {
        const size_t end = std::min(n, at + (size_t)kMaxPassElements);
        PassOp op;
        op.kick = first && kick;
        op.kappa = op.kick ? kappa : 0.0;
        op.els = pack(els, at, end);
        op.deposit = (end == n) && deposit;
        ops.push_back(op);
        first = false;
        at = end;
    } while (at < n);
}

// The line density, when on, goes with every pass that kicks or deposits.
scpic_status check_line(const scpic_ctx *c, const scpic_particles *p)
{
    if (c->line.nz == 0) return SCPIC_OK;
    if (!c->sw.pipe)
        return fail(SCPIC_EUNSUPPORTED, "the line density needs the grounded pipe solver (its "
                                        "longitudinal kick uses the absolute potential)");
    if (p->n > 0 && (!p->sigma || !p->psigma))
        return fail(SCPIC_EINVAL, "the line density needs the particles' sigma and psigma");
    if (p->w)
        return fail(SCPIC_EINVAL, "per-particle kick weights and the line density exclude each "
                                  "other (the line density computes the weights)");
    if (c->bspline)
        return fail(SCPIC_EUNSUPPORTED, "the line density takes the cloud-in-cell gather");
    // the per-workgroup line histogram counts 4096 per particle in 32 bits
    const int blocks = blocks_for(c, p->n, true);
    if (blocks > 0 && (p->n + blocks - 1) / blocks > (int64_t)(1 << 20) - 1024)
        return fail(SCPIC_EUNSUPPORTED, "the line density takes at most 2^20 particles per "
                                        "workgroup (raise SCPIC_OPT_PASS_BLOCKS)");
    return SCPIC_OK;
}

// per_element: a scpic_push / scpic_deposit / scpic_kick call, which stays
// transverse and gathers the field it is given (no line density, no B-spline
// field); the track and the fused pass take the context's modes.
scpic_status enqueue_pass(scpic_ctx *c, hipStream_t s, const scpic_particles *parts,
                          const PassOp &op, bool per_element = false)
{
    const int blocks = blocks_for(c, parts->n, op.deposit || op.kick);
    const LineSpec *line =
        !per_element && c->line.nz > 0 && (op.kick || op.deposit) ? &c->line : nullptr;
    const void *bphi = !per_element && c->bspline && op.kick ? c->sw.phi : nullptr;
    hipError_t e = launch_pass(s, to_ptrs(parts), c->geom, op.kick, c->mixed, c->ef, op.kappa,
                               op.els, op.deposit, c->dep, blocks, c->pass_threads, line, bphi);
    if (e != hipSuccess) return fail_hip(e, "particle pass launch");
    if (op.deposit) c->last_deposit_blocks = blocks;
    return SCPIC_OK;
}

scpic_status enqueue_grid_phase(scpic_ctx *c, hipStream_t s, double scale)
{
    hipError_t e = launch_solve_partials(s, c->sw, c->dep, c->last_deposit_blocks, scale, c->ef);
    if (e != hipSuccess) return fail_hip(e, "solve launch");
    return SCPIC_OK;
}

// Schedule of one turn.  The kick of a space-charge location is applied at
// the start of the next pass (positions are unchanged between the deposit and
// that kick, so this equals kicking at the location).  first_turn: no kick is
// pending from a previous turn and the trailing elements after the last SC
// location have not been pushed yet.
void build_turn(const std::vector<const scpic_element *> &all, bool first_turn,
                std::vector<PassOp> &ops, bool &any_sc, double &last_kappa,
                std::vector<const scpic_element *> &trailing)
{
    std::vector<size_t> sc;
    for (size_t i = 0; i < all.size(); ++i)
        if (all[i]->kind == SCPIC_EL_SC) sc.push_back(i);
    any_sc = !sc.empty();
    trailing.clear();
    if (!any_sc) {
        emit_segment(ops, false, 0.0, all, false);
        return;
    }
    for (size_t i = sc.back() + 1; i < all.size(); ++i) trailing.push_back(all[i]);
    last_kappa = all[sc.back()]->p[0];
    std::vector<const scpic_element *> seg;
    if (!first_turn) seg = trailing;
    for (size_t i = 0; i < sc[0]; ++i) seg.push_back(all[i]);
    emit_segment(ops, !first_turn, last_kappa, seg, true);
    for (size_t k = 1; k < sc.size(); ++k) {
        seg.clear();
        for (size_t i = sc[k - 1] + 1; i < sc[k]; ++i) seg.push_back(all[i]);
        emit_segment(ops, true, all[sc[k - 1]]->p[0], seg, true);
    }
}

scpic_status enqueue_ops(scpic_ctx *c, hipStream_t s, const scpic_particles *parts,
                         const std::vector<PassOp> &ops, double scale)
{
    for (const PassOp &op : ops) {
        scpic_status st = enqueue_pass(c, s, parts, op);
        if (st) return st;
        if (op.deposit) {
            st = enqueue_grid_phase(c, s, scale);
            if (st) return st;
        }
    }
    return SCPIC_OK;
}

std::vector<unsigned char> graph_key(const scpic_ctx *c, const scpic_particles *p,
                                     const std::vector<PassOp> &ops)
{
    std::vector<unsigned char> k;
    auto put = [&k](const void *d, size_t n) {
        const unsigned char *b = (const unsigned char *)d;
        k.insert(k.end(), b, b + n);
    };
    put(p, sizeof(*p));
    put(&c->pass_blocks, sizeof(c->pass_blocks));
    put(&c->pass_threads, sizeof(c->pass_threads));
    for (const PassOp &op : ops) {
        put(&op.kick, sizeof(op.kick));
        put(&op.kappa, sizeof(op.kappa));
        put(&op.deposit, sizeof(op.deposit));
        put(&op.els.n_el, sizeof(op.els.n_el));
        put(op.els.kind, sizeof(int32_t) * op.els.n_el);
        put(op.els.p, sizeof(double) * 16 * op.els.n_el);
    }
    return k;
}

scpic_status get_turn_graph(scpic_ctx *c, const scpic_particles *parts,
                            const std::vector<PassOp> &ops, double scale, hipGraphExec_t *out)
{
    std::vector<unsigned char> key = graph_key(c, parts, ops);
    key.insert(key.end(), (unsigned char *)&scale, (unsigned char *)&scale + sizeof(scale));
    for (auto &g : c->graphs)
        if (g.key == key) {
            g.last_use = ++c->use_counter;
            *out = g.exec;
            return SCPIC_OK;
        }
    if (!c->capture_stream) SCPIC_HIP_TRY(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking), "hipStreamCreate");
    SCPIC_HIP_TRY(hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal),
                  "hipStreamBeginCapture");
    const int saved_blocks = c->last_deposit_blocks;
    scpic_status st = enqueue_ops(c, c->capture_stream, parts, ops, scale);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(c->capture_stream, &graph);
    c->last_deposit_blocks = saved_blocks;
    if (st) {
        if (graph) hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail_hip(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) return fail_hip(e, "hipGraphInstantiate");
    if (c->graphs.size() >= 8) {
        auto it = std::min_element(c->graphs.begin(), c->graphs.end(),
                                   [](const GraphEntry &a, const GraphEntry &b) {
                                       return a.last_use < b.last_use;
                                   });
        hipGraphExecDestroy(it->exec);
        c->graphs.erase(it);
    }
    GraphEntry ge;
    ge.key = std::move(key);
    ge.exec = exec;
    ge.last_use = ++c->use_counter;
    c->graphs.push_back(std::move(ge));
    *out = exec;
    return SCPIC_OK;
}

// Free-space Green's function of lap G = -2 pi delta on node offsets, with
// the self-cell value replaced by the cell average of -ln r (from the
// antiderivative F of ln(x^2+y^2): int_0^a int_0^b = F(a, b)).
double green_offset(int di, int dj, double dx, double dy)
{
    if (di == 0 && dj == 0) {
        const double a = 0.5 * dx, b = 0.5 * dy;
        const double f = a * b * (std::log(a * a + b * b) - 3.0) + a * a * std::atan(b / a) +
                         b * b * std::atan(a / b);
        return -f / (2.0 * a * b);
    }
    const double X = di * dx, Y = dj * dy;
    return -0.5 * std::log(X * X + Y * Y);
}

}  // namespace

namespace scpic {

// Spectrum of the mx x my periodic kernel Gp(X, Y) = G(min(X, mx-X),
// min(Y, my-Y)) (mx >= 2 nx, my >= 2 ny).  Gp is even in both offsets, so its
// DFT is the real cosine sum; it is taken separably (over Y, then X) and
// divided by mx*my, the normalisation of the unnormalised inverse
// transforms.  Layout [my/2+1][mx].
void green_spectrum_host(int mx, int my, double dx, double dy, double *ghat_t)
{
    const int ny = my / 2;  // the half spectrum's last column
    std::vector<double> cxs(mx), cys(my), gp((size_t)mx * my), h((size_t)mx * (ny + 1));
    for (int t = 0; t < mx; ++t) cxs[t] = std::cos(2.0 * M_PI * t / mx);
    for (int t = 0; t < my; ++t) cys[t] = std::cos(2.0 * M_PI * t / my);
    for (int X = 0; X < mx; ++X)
        for (int Y = 0; Y < my; ++Y)
            gp[(size_t)X * my + Y] = green_offset(std::min(X, mx - X), std::min(Y, my - Y), dx, dy);
    for (int X = 0; X < mx; ++X)
        for (int l = 0; l <= ny; ++l) {
            double s = 0.0;
            for (int Y = 0; Y < my; ++Y) s += gp[(size_t)X * my + Y] * cys[((size_t)l * Y) % my];
            h[(size_t)X * (ny + 1) + l] = s;
        }
    const double norm = 1.0 / ((double)mx * (double)my);
    for (int l = 0; l <= ny; ++l)
        for (int k = 0; k < mx; ++k) {
            double s = 0.0;
            for (int X = 0; X < mx; ++X) s += h[(size_t)X * (ny + 1) + l] * cxs[((size_t)k * X) % mx];
            ghat_t[(size_t)l * mx + k] = s * norm;
        }
}

// Grounded rectangular pipe (walls through node 0 and node n of each axis):
// the odd extension of the charge is 2nx x 2ny periodic, and the 5-point
// Laplacian acts on its DFT mode (k, l) as multiplication by
//   lambda = -4 (sin^2(pi k / mx) / dx^2 + sin^2(pi l / my) / dy^2).
// With the open-boundary solve's normalisation (lap phi = -2 pi rho per unit
// area) the potential's spectrum is -2 pi rho^ / (dx dy lambda); mode (0, 0)
// is zero (the odd extension has no mean).  Divided by mx*my like ghat_t.
void pipe_spectrum_host(int nx, int ny, double dx, double dy, double *ghat_t)
{
    const int mx = 2 * nx, my = 2 * ny;
    const double norm = 1.0 / ((double)mx * (double)my);
    for (int l = 0; l <= ny; ++l)
        for (int k = 0; k < mx; ++k) {
            const double sk = std::sin(M_PI * k / mx), sl = std::sin(M_PI * l / my);
            const double lam = -4.0 * (sk * sk / (dx * dx) + sl * sl / (dy * dy));
            ghat_t[(size_t)l * mx + k] =
                (k == 0 && l == 0) ? 0.0 : (-2.0 * M_PI / (dx * dy)) / lam * norm;
        }
}

}  // namespace scpic

namespace {

// Green's spectrum (open boundary) or the pipe's mode divisors, twiddles and
// difference factors of a grid, converted to T and copied to the given
// device tables (the twiddle tables laid out as SolveWorkspace's stw_x and
// stw_y: the stage tables hold the plain tables' values, so every FFT
// multiplies by exactly the twiddles of a plain table).
// The pipe needs mx = 2 nx and my = 2 ny (its walls sit at node 0 and node
// n of each axis); the open boundary takes the padded lengths of fft_len.
template <typename T>
scpic_status upload_grid_tables(const scpic_grid &grid, void *ghat_t, void *stw_x, void *stw_y,
                                void *sx_t, void *sy_t, bool pipe = false)
{
    const int nx = grid.nx, ny = grid.ny, mx = fft_len(nx), my = fft_len(ny), hy = my / 2;
    std::vector<double> ghat((size_t)(hy + 1) * mx);
    if (pipe)
        pipe_spectrum_host(nx, ny, grid.dx, grid.dy, ghat.data());
    else
        green_spectrum_host(mx, my, grid.dx, grid.dy, ghat.data());
    std::vector<T> g_t(ghat.size()), twx(2 * (size_t)mx), twy(2 * (size_t)my), sx(mx), sy(hy + 1);
    for (size_t i = 0; i < ghat.size(); ++i) g_t[i] = (T)ghat[i];
    for (int t = 0; t < mx; ++t) {
        twx[2 * t] = (T)std::cos(2.0 * M_PI * t / mx);
        twx[2 * t + 1] = (T)(-std::sin(2.0 * M_PI * t / mx));
        sx[t] = (T)(std::sin(2.0 * M_PI * t / mx) / grid.dx);
    }
    for (int t = 0; t < my; ++t) {
        twy[2 * t] = (T)std::cos(2.0 * M_PI * t / my);
        twy[2 * t + 1] = (T)(-std::sin(2.0 * M_PI * t / my));
    }
    for (int l = 0; l <= hy; ++l) sy[l] = (T)(std::sin(2.0 * M_PI * l / my) / grid.dy);
    SCPIC_HIP_TRY(hipMemcpy(ghat_t, g_t.data(), sizeof(T) * g_t.size(), hipMemcpyHostToDevice), "upload ghat");
    const int lx = ilog2(mx), ly = ilog2(my);
    std::vector<T> stx(2 * (size_t)mx, T(0)), sty(2 * (size_t)(2 * my + 1), T(0));
    for (int e = 0; e < stage_twiddle_count(mx, lx); ++e) {
        const int t = stage_twiddle_exponent(e, mx, lx);
        stx[2 * e] = twx[2 * t];
        stx[2 * e + 1] = twx[2 * t + 1];
    }
    for (int l = 0; l <= hy; ++l) {
        sty[2 * l] = twy[2 * l];
        sty[2 * l + 1] = twy[2 * l + 1];
    }
    for (int e = 0; e < stage_twiddle_count(hy, ly - 1); ++e) {
        const int t = 2 * stage_twiddle_exponent(e, hy, ly - 1);
        sty[2 * (hy + 1 + e)] = twy[2 * t];
        sty[2 * (hy + 1 + e) + 1] = twy[2 * t + 1];
    }
    for (int e = 0; e < stage_twiddle_count(my, ly); ++e) {
        const int t = stage_twiddle_exponent(e, my, ly);
        sty[2 * (my + 1 + e)] = twy[2 * t];
        sty[2 * (my + 1 + e) + 1] = twy[2 * t + 1];
    }
    SCPIC_HIP_TRY(hipMemcpy(stw_x, stx.data(), sizeof(T) * stx.size(), hipMemcpyHostToDevice), "upload twiddles");
    SCPIC_HIP_TRY(hipMemcpy(stw_y, sty.data(), sizeof(T) * sty.size(), hipMemcpyHostToDevice), "upload twiddles");
    SCPIC_HIP_TRY(hipMemcpy(sx_t, sx.data(), sizeof(T) * sx.size(), hipMemcpyHostToDevice), "upload sx");
    SCPIC_HIP_TRY(hipMemcpy(sy_t, sy.data(), sizeof(T) * sy.size(), hipMemcpyHostToDevice), "upload sy");
    return SCPIC_OK;
}

template <typename T>
scpic_status upload_tables(scpic_ctx *c)
{
    return upload_grid_tables<T>(c->grid, c->sw.ghat_t, c->sw.stw_x, c->sw.stw_y, c->sw.sx,
                                 c->sw.sy, c->sw.pipe);
}

scpic_status create_impl(scpic_ctx *c, const scpic_grid *grid, int32_t precision, void *stream)
{
    c->grid = *grid;
    c->mixed = precision == SCPIC_MIXED;
    c->stream = (hipStream_t)stream;
    c->geom.nx = grid->nx;
    c->geom.ny = grid->ny;
    c->geom.x_min = grid->x_min;
    c->geom.y_min = grid->y_min;
    c->geom.inv_dx = 1.0 / grid->dx;
    c->geom.inv_dy = 1.0 / grid->dy;
    SCPIC_HIP_TRY(hipGetDevice(&c->device), "hipGetDevice");
    hipDeviceProp_t prop;
    SCPIC_HIP_TRY(hipGetDeviceProperties(&prop, c->device), "hipGetDeviceProperties");
    c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
    c->max_blocks = std::min(2 * c->n_cu, kMaxPassBlocks);
    const int nx = grid->nx, ny = grid->ny, ncell = nx * ny;
    const size_t lds = sizeof(uint32_t) * (size_t)ncell;
    (void)lds;
    const size_t fe = field_elem_size(c);
    const size_t ce = 2 * fe;
    scpic_status st;
    void *p;
#define ALLOC(dst, bytes)                               \
    do {                                                \
        if ((st = dev_alloc(c, &p, (bytes)))) return st; \
        dst = decltype(dst)(p);                         \
    } while (0)
    ALLOC(c->dep.partial, sizeof(uint32_t) * (size_t)c->max_blocks * ncell);
    ALLOC(c->dep.header, sizeof(BlockHeader) * (size_t)c->max_blocks);
    ALLOC(c->dep.carry, sizeof(unsigned long long) * (size_t)ncell);
    c->dep.max_blocks = c->max_blocks;
    c->sw.nx = nx;
    c->sw.ny = ny;
    const int mx = fft_len(nx), my = fft_len(ny), hy = my / 2;
    c->sw.mx = mx;
    c->sw.my = my;
    c->sw.log2_mx = ilog2(mx);
    c->sw.log2_my = ilog2(my);
    c->sw.mixed = c->mixed;
    c->sw.pipe = false;
    ALLOC(c->sw.stw_x, ce * mx);
    ALLOC(c->sw.stw_y, ce * (2 * (size_t)my + 1));
    ALLOC(c->sw.ghat_t, fe * (size_t)(hy + 1) * mx);
    ALLOC(c->sw.sx, fe * mx);
    ALLOC(c->sw.sy, fe * (hy + 1));
    ALLOC(c->sw.spec_a, ce * (size_t)(hy + 1) * nx);
    ALLOC(c->sw.spec_bx, ce * (size_t)(hy + 1) * nx);
    ALLOC(c->sw.spec_by, ce * (size_t)(hy + 1) * nx);
    ALLOC(c->ef, 2 * fe * ncell);
    ALLOC(c->diag_part, sizeof(double) * kMomentBlocks * kMoments);
    ALLOC(c->diag_sums, sizeof(double) * 2 * kMoments);
#undef ALLOC
    SCPIC_HIP_TRY(hipMemset(c->dep.carry, 0, sizeof(unsigned long long) * ncell), "hipMemset");
    // headers start "unknown" (all -1): the first deposit uses the whole grid
    // as its LDS tile when it fits
    SCPIC_HIP_TRY(hipMemset(c->dep.header, 0xff, sizeof(BlockHeader) * c->max_blocks), "hipMemset");
    SCPIC_HIP_TRY(hipMemset(c->ef, 0, 2 * fe * ncell), "hipMemset");
    st = c->mixed ? upload_tables<float>(c) : upload_tables<double>(c);
    if (st) return st;
    // the pass's static LDS is a few words; keep 256 bytes for it
    SCPIC_HIP_TRY(prepare_pass_kernels(prop.sharedMemPerBlock), "hipFuncSetAttribute");
    SCPIC_HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    return SCPIC_OK;
}

}  // namespace

extern "C" {

int32_t scpic_version(void) { return 200; }

const char *scpic_last_error(void) { return g_last_error.c_str(); }

scpic_status scpic_create(scpic_ctx **out, const scpic_grid *grid, int32_t precision,
                          void *hip_stream)
{
    g_last_error.clear();
    if (!out) return fail(SCPIC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!grid) return fail(SCPIC_EINVAL, "grid is NULL");
    if (precision != SCPIC_FP64 && precision != SCPIC_MIXED)
        return fail(SCPIC_EINVAL, "precision must be SCPIC_FP64 or SCPIC_MIXED");
    if (scpic_status st = check_grid(grid)) return st;
    scpic_ctx *c = new (std::nothrow) scpic_ctx();
    if (!c) return fail(SCPIC_ENOMEM, "host allocation failed");
    scpic_status st = create_impl(c, grid, precision, hip_stream);
    if (st) {
        free_all(c);
        delete c;
        return st;
    }
    *out = c;
    return SCPIC_OK;
}

scpic_status scpic_destroy(scpic_ctx *ctx)
{
    g_last_error.clear();
    if (!ctx) return SCPIC_OK;
    hipStreamSynchronize(ctx->stream);
    free_all(ctx);
    delete ctx;
    return SCPIC_OK;
}

scpic_status scpic_set_stream(scpic_ctx *ctx, void *hip_stream)
{
    g_last_error.clear();
    if (scpic_status st = check_ctx(ctx)) return st;
    ctx->stream = (hipStream_t)hip_stream;
    return SCPIC_OK;
}

scpic_status scpic_set_option(scpic_ctx *ctx, int32_t option, int64_t value)
{
    g_last_error.clear();
    if (scpic_status st = check_ctx(ctx)) return st;
    switch (option) {
    case SCPIC_OPT_USE_GRAPH:
        ctx->use_graph = value != 0;
        return SCPIC_OK;
    case SCPIC_OPT_PASS_BLOCKS:
        if (value < 0 || value > ctx->max_blocks)
            return fail(SCPIC_EINVAL, "pass blocks must be in [0, " + std::to_string(ctx->max_blocks) + "]");
        ctx->pass_blocks = (int)value;
        return SCPIC_OK;
    case SCPIC_OPT_SOLVER: {
        if (value != SCPIC_SOLVER_OPEN && value != SCPIC_SOLVER_PIPE)
            return fail(SCPIC_EINVAL, "solver must be SCPIC_SOLVER_OPEN or SCPIC_SOLVER_PIPE");
        const bool pipe = value == SCPIC_SOLVER_PIPE;
        if (pipe == ctx->sw.pipe) return SCPIC_OK;
        if (pipe && !(is_pow2(ctx->grid.nx) && is_pow2(ctx->grid.ny)))
            return fail(SCPIC_EUNSUPPORTED, "the grounded pipe needs nx and ny powers of two (its "
                                            "odd extension has length 2n, a radix-2/4 FFT length)");
        // captured turns carry the solver: drop them once queued work is done
        SCPIC_HIP_TRY(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        for (auto &g : ctx->graphs)
            if (g.exec) hipGraphExecDestroy(g.exec);
        ctx->graphs.clear();
        ctx->sw.pipe = pipe;
        return ctx->mixed ? upload_tables<float>(ctx) : upload_tables<double>(ctx);
    }
    case SCPIC_OPT_GATHER: {
        if (value != SCPIC_GATHER_CIC && value != SCPIC_GATHER_BSPLINE)
            return fail(SCPIC_EINVAL, "gather must be SCPIC_GATHER_CIC or SCPIC_GATHER_BSPLINE");
        const bool bs = value == SCPIC_GATHER_BSPLINE;
        if (bs == ctx->bspline) return SCPIC_OK;
        SCPIC_HIP_TRY(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        drop_graphs(ctx);
        if (bs)
            if (scpic_status st = ensure_potential(ctx)) return st;
        ctx->bspline = bs;
        ctx->sw.want_phi = bs || ctx->line.nz > 0;
        return SCPIC_OK;
    }
    case SCPIC_OPT_PASS_THREADS:
        if (value != 256 && value != 512 && value != 1024)
            return fail(SCPIC_EINVAL, "pass threads must be 256, 512 or 1024");
        ctx->pass_threads = (int)value;
        return SCPIC_OK;
    default:
        return fail(SCPIC_EINVAL, "unknown option " + std::to_string(option));
    }
}

scpic_status scpic_push(scpic_ctx *ctx, const scpic_particles *parts,
                        const scpic_element *elements, int32_t n_el)
{
    g_last_error.clear();
    if (scpic_status st = check_ctx(ctx)) return st;
    if (scpic_status st = check_parts(parts)) return st;
    std::vector<const scpic_element *> els;
    if (scpic_status st = collect_elements(elements, n_el, els, false)) return st;
    if (scpic_status st = check_longitudinal(els, parts)) return st;
    if (els.empty() || parts->n == 0) return SCPIC_OK;
    std::vector<PassOp> ops;
    emit_segment(ops, false, 0.0, els, false);
    for (const PassOp &op : ops)
        if (scpic_status st = enqueue_pass(ctx, ctx->stream, parts, op, true)) return st;
    return SCPIC_OK;
}

scpic_status scpic_deposit(scpic_ctx *ctx, const scpic_particles *parts, int64_t *rho,
                           int64_t *n_in)
{
    g_last_error.clear();
    if (scpic_status st = check_ctx(ctx)) return st;
    if (scpic_status st = check_parts(parts)) return st;
    if (!rho) return fail(SCPIC_EINVAL, "rho is NULL");
    PassOp op;
    std::memset(&op, 0, sizeof(op));
    op.deposit = true;
    if (scpic_status st = enqueue_pass(ctx, ctx->stream, parts, op, true)) return st;
    const int blocks = parts->n > 0 ? ctx->last_deposit_blocks : 0;
    hipError_t e = launch_reduce(ctx->stream, ctx->dep, blocks, ctx->grid.nx, ctx->grid.ny, rho, n_in);
    if (e != hipSuccess) return fail_hip(e, "reduce launch");
    return SCPIC_OK;
}

scpic_status scpic_solve(scpic_ctx *ctx, const int64_t *rho, double scale, void *ex, void *ey)
{
    g_last_error.clear();
    if (scpic_status st = check_ctx(ctx)) return st;
    if (!rho || !ex || !ey) return fail(SCPIC_EINVAL, "rho, ex and ey must be non-NULL");
    if (!std::isfinite(scale)) return fail(SCPIC_EINVAL, "scale must be finite");
    hipError_t e = launch_solve(ctx->stream, ctx->sw, rho, scale, ex, ey, nullptr);
    if (e != hipSuccess) return fail_hip(e, "solve launch");
    return SCPIC_OK;
}

scpic_status scpic_kick(scpic_ctx *ctx, const scpic_particles *parts, const void *ex,
                        const void *ey, double kappa)
{
    g_last_error.clear();
    if (scpic_status st = check_ctx(ctx)) return st;
    if (scpic_status st = check_parts(parts)) return st;
    if (!ex || !ey) return fail(SCPIC_EINVAL, "ex and ey must be non-NULL");
    if (!std::isfinite(kappa)) return fail(SCPIC_EINVAL, "kappa must be finite");
    PassOp op;
    std::memset(&op, 0, sizeof(op));
    op.kick = true;
    op.kappa = kappa;
    hipError_t e = launch_interleave(ctx->stream, ctx->mixed, true, (void *)ex, (void *)ey, ctx->ef,
                                     ctx->grid.nx * ctx->grid.ny);
    if (e != hipSuccess) return fail_hip(e, "field interleave launch");
    return enqueue_pass(ctx, ctx->stream, parts, op, true);
}

scpic_status scpic_pass(scpic_ctx *ctx, const scpic_particles *parts, int32_t kick, double kappa,
                        const scpic_element *elements, int32_t n_el, int32_t deposit)
{
    g_last_error.clear();
    if (scpic_status st = check_ctx(ctx)) return st;
    if (scpic_status st = check_parts(parts)) return st;
    if (n_el > kMaxPassElements) return fail(SCPIC_EINVAL, "at most 12 elements per pass");
    std::vector<const scpic_element *> els;
    if (scpic_status st = collect_elements(elements, n_el, els, true)) return st;
    for (auto *e : els)
        if (e->kind == SCPIC_EL_SC) return fail(SCPIC_EINVAL, "a pass takes no SC element");
    if (scpic_status st = check_longitudinal(els, parts)) return st;
    if (kick || deposit)
        if (scpic_status st = check_line(ctx, parts)) return st;
    PassOp op;
    op.kick = kick != 0;
    op.kappa = kappa;
    op.els = pack(els, 0, els.size());
    op.deposit = deposit != 0;
    return enqueue_pass(ctx, ctx->stream, parts, op);
}

scpic_status scpic_reduce_solve(scpic_ctx *ctx, double scale)
{
    g_last_error.clear();
    if (scpic_status st = check_ctx(ctx)) return st;
    return enqueue_grid_phase(ctx, ctx->stream, scale);
}

scpic_status scpic_get_field(scpic_ctx *ctx, void *ex, void *ey)
{
    g_last_error.clear();
    if (scpic_status st = check_ctx(ctx)) return st;
    if (!ex || !ey) return fail(SCPIC_EINVAL, "ex and ey must be non-NULL");
    hipError_t e = launch_interleave(ctx->stream, ctx->mixed, false, ex, ey, ctx->ef,
                                     ctx->grid.nx * ctx->grid.ny);
    if (e != hipSuccess) return fail_hip(e, "field copy launch");
    return SCPIC_OK;
}

scpic_status scpic_set_line_density(scpic_ctx *ctx, int32_t nz, double z_min, double dz,
                                    double gamma0)
{
    g_last_error.clear();
    if (scpic_status st = check_ctx(ctx)) return st;
    if (nz != 0 && (nz < 8 || nz > kMaxLineNodes))
        return fail(SCPIC_EINVAL, "nz must be 0 or in [8, " + std::to_string(kMaxLineNodes) + "]");
    if (nz != 0 && !(dz > 0.0 && std::isfinite(dz) && std::isfinite(z_min) &&
                     std::isfinite(gamma0) && gamma0 >= 1.0))
        return fail(SCPIC_EINVAL, "dz must be positive and finite, z_min finite, gamma0 >= 1");
    // captured turns carry the line: drop them once queued work is done
    SCPIC_HIP_TRY(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    drop_graphs(ctx);
    free_line(ctx);
    if (nz == 0) return SCPIC_OK;
    if (scpic_status st = ensure_potential(ctx)) return st;
    const size_t sizes[2] = {sizeof(unsigned long long) * (size_t)ctx->max_blocks * nz,
                             sizeof(double) * 2 * (size_t)nz};
    void *mem[2] = {};
    for (int k = 0; k < 2; ++k) {
        hipError_t e = hipMalloc(&mem[k], sizes[k]);
        if (e != hipSuccess) {
            for (int j = 0; j < k; ++j) hipFree(mem[j]);
            return fail(SCPIC_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
        }
    }
    for (int k = 0; k < 2; ++k) ctx->line_mem.push_back(mem[k]);
    // a kick before the first deposit sees an empty line (no kick)
    SCPIC_HIP_TRY(hipMemset(mem[1], 0, sizes[1]), "hipMemset");
    LineSpec &L = ctx->line;
    L.nz = nz;
    L.z_min = z_min;
    L.dz = dz;
    L.inv_dz = 1.0 / dz;
    L.gamma0 = gamma0;
    L.partial = (unsigned long long *)mem[0];
    L.lw = (double *)mem[1];
    L.ld = L.lw + nz;
    L.phi = ctx->sw.phi;
    ctx->sw.line = L;
    ctx->sw.want_phi = true;
    return SCPIC_OK;
}

scpic_status scpic_get_potential(scpic_ctx *ctx, void *phi)
{
    g_last_error.clear();
    if (scpic_status st = check_ctx(ctx)) return st;
    if (!phi) return fail(SCPIC_EINVAL, "phi is NULL");
    if (!ctx->sw.want_phi)
        return fail(SCPIC_EINVAL, "the potential is kept only with the line density or the "
                                  "B-spline gather");
    SCPIC_HIP_TRY(hipMemcpyAsync(phi, ctx->sw.phi,
                                 field_elem_size(ctx) * (size_t)(ctx->grid.nx + 2) *
                                     (ctx->grid.ny + 2),
                                 hipMemcpyDeviceToDevice, ctx->stream),
                  "hipMemcpyAsync");
    return SCPIC_OK;
}

scpic_status scpic_get_line_state(scpic_ctx *ctx, double *lw, double *ld)
{
    g_last_error.clear();
    if (scpic_status st = check_ctx(ctx)) return st;
    if (ctx->line.nz == 0) return fail(SCPIC_EINVAL, "the line density is off");
    if (lw)
        SCPIC_HIP_TRY(hipMemcpyAsync(lw, ctx->line.lw, sizeof(double) * ctx->line.nz,
                                     hipMemcpyDeviceToDevice, ctx->stream),
                      "hipMemcpyAsync");
    if (ld)
        SCPIC_HIP_TRY(hipMemcpyAsync(ld, ctx->line.ld, sizeof(double) * ctx->line.nz,
                                     hipMemcpyDeviceToDevice, ctx->stream),
                      "hipMemcpyAsync");
    return SCPIC_OK;
}

static scpic_status track_impl(scpic_ctx *ctx, const scpic_particles *parts,
                               const scpic_element *turn, int32_t n_el, int32_t n_turns);

scpic_status scpic_diagnose(scpic_ctx *ctx, const scpic_particles *parts, scpic_diag *out)
{
    g_last_error.clear();
    if (scpic_status st = check_ctx(ctx)) return st;
    if (scpic_status st = check_parts(parts)) return st;
    if (!out) return fail(SCPIC_EINVAL, "out is NULL");
    *out = scpic_diag{};
    if (parts->n == 0) return SCPIC_OK;
    SCPIC_HIP_TRY(launch_moments(ctx->stream, to_ptrs(parts), ctx->diag_part, ctx->diag_sums),
                  "moments launch");
    double s[2 * kMoments];
    SCPIC_HIP_TRY(hipMemcpyAsync(s, ctx->diag_sums, sizeof(s), hipMemcpyDeviceToHost, ctx->stream),
                  "hipMemcpyAsync");
    SCPIC_HIP_TRY(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    const double a = s[0];
    if (!(a > 0.0)) return SCPIC_OK;
    out->alive = (int64_t)a;
    for (int k = 0; k < 4; ++k) out->mean[k] = s[1 + k] / a;
    const double *c = s + kMoments;
    const double ex = (c[0] / a) * (c[1] / a) - (c[2] / a) * (c[2] / a);
    const double ey = (c[3] / a) * (c[4] / a) - (c[5] / a) * (c[5] / a);
    out->emit_x = ex > 0.0 ? std::sqrt(ex) : 0.0;
    out->emit_y = ey > 0.0 ? std::sqrt(ey) : 0.0;
    return SCPIC_OK;
}

scpic_status scpic_track(scpic_ctx *ctx, const scpic_particles *parts, const scpic_element *turn,
                         int32_t n_el, int32_t n_turns, scpic_diag *diag)
{
    const scpic_status st = track_impl(ctx, parts, turn, n_el, n_turns);
    if (st || !diag) return st;
    return scpic_diagnose(ctx, parts, diag);
}

// scpic_track without the diagnostics.
static scpic_status track_impl(scpic_ctx *ctx, const scpic_particles *parts,
                               const scpic_element *turn, int32_t n_el, int32_t n_turns)
{
    g_last_error.clear();
    if (scpic_status st = check_ctx(ctx)) return st;
    if (scpic_status st = check_parts(parts)) return st;
    if (n_turns < 0) return fail(SCPIC_EINVAL, "n_turns is negative");
    std::vector<const scpic_element *> all;
    if (scpic_status st = collect_elements(turn, n_el, all, true)) return st;
    if (scpic_status st = check_longitudinal(all, parts)) return st;
    for (const scpic_element *e : all)
        if (e->kind == SCPIC_EL_SC) {
            if (scpic_status st = check_line(ctx, parts)) return st;
            break;
        }
    if (n_turns == 0 || all.empty() || parts->n == 0) return SCPIC_OK;
    const double scale = 1.0 / (kChargeOne * (double)parts->n);

    std::vector<PassOp> first, steady;
    std::vector<const scpic_element *> trailing;
    bool any_sc = false;
    double last_kappa = 0.0;
    build_turn(all, true, first, any_sc, last_kappa, trailing);
    if (!any_sc) {
        for (int t = 0; t < n_turns; ++t)
            if (scpic_status st = enqueue_ops(ctx, ctx->stream, parts, first, scale)) return st;
        return SCPIC_OK;
    }
    build_turn(all, false, steady, any_sc, last_kappa, trailing);
    if (scpic_status st = enqueue_ops(ctx, ctx->stream, parts, first, scale)) return st;
    if (n_turns > 1) {
        if (ctx->use_graph) {
            hipGraphExec_t exec = nullptr;
            if (scpic_status st = get_turn_graph(ctx, parts, steady, scale, &exec)) return st;
            for (int t = 1; t < n_turns; ++t)
                SCPIC_HIP_TRY(hipGraphLaunch(exec, ctx->stream), "hipGraphLaunch");
            // the graph's last depositing pass used the same block count
            for (const PassOp &op : steady)
                if (op.deposit) ctx->last_deposit_blocks = blocks_for(ctx, parts->n, true);
        } else {
            for (int t = 1; t < n_turns; ++t)
                if (scpic_status st = enqueue_ops(ctx, ctx->stream, parts, steady, scale)) return st;
        }
    }
    // epilogue: the last location's kick, then the elements after it
    std::vector<PassOp> tail;
    emit_segment(tail, true, last_kappa, trailing, false);
    return enqueue_ops(ctx, ctx->stream, parts, tail, scale);
}

}  // extern "C"

// ---- batches of independent beams -----------------------------------------

namespace {

// Device step tables of one schedule (the op list shared by every beam) and,
// for the steady turn, its captured graph.
struct BatchSchedule {
    std::vector<unsigned char> key;
    std::vector<PassOp> shape;     // kick / deposit per op (kappa, els unused)
    std::vector<char> six;         // per op: some beam's elements are thick
    BatchStep *steps = nullptr;    // device [n_ops][n_inst]
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
};

constexpr size_t kMaxSchedules = 16;

}  // namespace

struct scpic_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    bool mixed = false;
    int n_cu = 0;
    int n_inst = 0;
    int pass_threads = 1024;  // launch shape of the batched pass (autotuned)
    int blocks_per_cu = 1;
    std::vector<int64_t> offsets;
    std::vector<int> max_slices;      // partial slices allocated per beam
    uint16_t *pass_table = nullptr;   // device, sized for the largest shape
    std::vector<scpic_grid> grids;
    std::vector<BatchInstance> inst;  // host copy of the device table
    BatchLaunch launch{};
    int total_pass_blocks = 0, total_rows = 0, total_cols = 0, max_mx = 0, max_ny = 0, max_my = 0;
    int max_beam_blocks = 0;  // most pass workgroups of one beam in the current layout
    std::vector<void *> allocations;
    std::vector<BatchSchedule> schedules;
    uint64_t use_counter = 0;
};

namespace {

scpic_status batch_alloc(scpic_batch *b, void **p, size_t bytes)
{
    hipError_t e = hipMalloc(p, bytes ? bytes : 1);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(SCPIC_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    b->allocations.push_back(*p);
    return SCPIC_OK;
}

void batch_drop_schedule(BatchSchedule &s)
{
    if (s.exec) hipGraphExecDestroy(s.exec);
    if (s.steps) hipFree(s.steps);
    s.exec = nullptr;
    s.steps = nullptr;
}

void batch_free_all(scpic_batch *b)
{
    for (auto &s : b->schedules) batch_drop_schedule(s);
    b->schedules.clear();
    for (void *p : b->allocations) hipFree(p);
    b->allocations.clear();
    if (b->capture_stream) hipStreamDestroy(b->capture_stream);
    b->capture_stream = nullptr;
}

// Upper bound of beam k's workgroups in a batched pass of `slots`
// workgroups: its proportional share rounded up, at most one per `threads`
// particles, at least one for a non-empty beam (sizes the partial slices).
int batch_pass_blocks(int64_t n_k, int64_t total, int64_t slots, int threads)
{
    if (n_k <= 0) return 0;
    const int64_t share = (n_k * slots + total - 1) / total;
    const int64_t need = (n_k + threads - 1) / threads;
    return (int)std::max<int64_t>(1, std::min<int64_t>({share, need, (int64_t)kMaxPassBlocks}));
}

// Workgroups per beam for a batched pass of about `slots` workgroups in all:
// one per non-empty beam, then each further workgroup to the beam with the
// most particles per workgroup (which minimises the largest workgroup's
// share, so the pass ends with one round of equal workgroups), within the
// caps (one per `threads` particles, the allocated slices).
std::vector<int> batch_assign_blocks(const std::vector<int64_t> &n, int64_t slots, int threads,
                                     const std::vector<int> &cap)
{
    const size_t k_n = n.size();
    std::vector<int> blocks(k_n, 0);
    int64_t used = 0;
    for (size_t k = 0; k < k_n; ++k)
        if (n[k] > 0) {
            blocks[k] = 1;
            ++used;
        }
    while (used < slots) {
        size_t best = k_n;
        double best_load = 0.0;
        for (size_t k = 0; k < k_n; ++k) {
            if (blocks[k] == 0 || blocks[k] >= cap[k]) continue;
            if ((int64_t)blocks[k] * threads >= n[k]) continue;
            const double load = (double)n[k] / blocks[k];
            if (load > best_load) {
                best_load = load;
                best = k;
            }
        }
        if (best == k_n) break;
        ++blocks[best];
        ++used;
    }
    return blocks;
}

// Candidate launch shapes of the batched pass (threads per workgroup,
// workgroups per compute unit); the largest allocation covers them all.
constexpr int kTuneThreads[] = {256, 512, 1024};
constexpr int kTuneBlocksPerCu[] = {1, 2, 4};
constexpr int kMinTuneThreads = 256, kMaxTuneBlocksPerCu = 4;

// Lay the batched pass out for a launch shape: each beam's workgroups and the
// workgroup -> beam table, uploaded with the beam table.  Headers restart as
// "unknown" (their boxes belonged to the previous assignment of particles).
scpic_status batch_layout(scpic_batch *b, int threads, int blocks_per_cu)
{
    std::vector<int64_t> sizes(b->n_inst);
    for (int k = 0; k < b->n_inst; ++k) sizes[k] = b->inst[k].n;
    const std::vector<int> blocks =
        batch_assign_blocks(sizes, (int64_t)b->n_cu * blocks_per_cu, threads, b->max_slices);
    // Workgroups are dispatched in index order as compute units free up, so
    // the beams whose workgroups carry the most particles go first and the
    // lightest fill the end of the launch (longest first keeps the tail short).
    // A beam's workgroups stay contiguous; results do not depend on the order.
    std::vector<int> order(b->n_inst);
    for (int k = 0; k < b->n_inst; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int u, int v) {
        const double lu = blocks[u] ? (double)sizes[u] / blocks[u] : 0.0;
        const double lv = blocks[v] ? (double)sizes[v] / blocks[v] : 0.0;
        return lu > lv;
    });
    std::vector<uint16_t> pass_inst;
    b->total_pass_blocks = 0;
    b->max_beam_blocks = 0;
    for (int k : order) {
        BatchInstance &I = b->inst[k];
        I.pass_blocks = blocks[k];
        I.pass_block0 = b->total_pass_blocks;
        b->total_pass_blocks += I.pass_blocks;
        b->max_beam_blocks = std::max(b->max_beam_blocks, I.pass_blocks);
        for (int t = 0; t < I.pass_blocks; ++t) pass_inst.push_back((uint16_t)k);
        SCPIC_HIP_TRY(hipMemsetAsync(I.dep.header, 0xff, sizeof(BlockHeader) * I.dep.max_blocks, b->stream), "hipMemsetAsync");
    }
    b->pass_threads = threads;
    b->blocks_per_cu = blocks_per_cu;
    SCPIC_HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    SCPIC_HIP_TRY(hipMemcpy((void *)b->launch.inst, b->inst.data(), sizeof(BatchInstance) * b->n_inst, hipMemcpyHostToDevice), "upload beams");
    if (!pass_inst.empty())
        SCPIC_HIP_TRY(hipMemcpy(b->pass_table, pass_inst.data(), sizeof(uint16_t) * pass_inst.size(), hipMemcpyHostToDevice), "upload tables");
    return SCPIC_OK;
}

struct GridTables {
    scpic_grid grid;
    void *ghat_t, *stw_x, *stw_y, *sx, *sy;
};

scpic_status batch_create_impl(scpic_batch *b, const scpic_grid *grids, const int64_t *offsets,
                               int n_inst, int32_t precision, void *stream)
{
    b->mixed = precision == SCPIC_MIXED;
    b->stream = (hipStream_t)stream;
    b->n_inst = n_inst;
    b->offsets.assign(offsets, offsets + n_inst + 1);
    b->grids.assign(grids, grids + n_inst);
    SCPIC_HIP_TRY(hipGetDevice(&b->device), "hipGetDevice");
    hipDeviceProp_t prop;
    SCPIC_HIP_TRY(hipGetDeviceProperties(&prop, b->device), "hipGetDeviceProperties");
    b->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
    const size_t fe = b->mixed ? sizeof(float) : sizeof(double), ce = 2 * fe;
    const int64_t total = offsets[n_inst];
    std::vector<GridTables> tables;
    std::vector<uint16_t> row_inst, col_inst;
    size_t pass_table_len = 0;
    b->inst.resize(n_inst);
    b->max_slices.resize(n_inst);
    scpic_status st;
    void *p;
#define BALLOC(dst, bytes)                                  \
    do {                                                    \
        if ((st = batch_alloc(b, &p, (bytes)))) return st;  \
        dst = decltype(dst)(p);                             \
    } while (0)
    for (int k = 0; k < n_inst; ++k) {
        const scpic_grid &gr = grids[k];
        const int nx = gr.nx, ny = gr.ny, ncell = nx * ny;
        const int64_t n_k = offsets[k + 1] - offsets[k];
        BatchInstance &I = b->inst[k];
        std::memset(&I, 0, sizeof(I));
        I.p0 = offsets[k];
        I.n = n_k;
        // enough partial slices for every candidate launch shape
        b->max_slices[k] = std::max(
            1, batch_pass_blocks(n_k, total, (int64_t)b->n_cu * kMaxTuneBlocksPerCu, kMinTuneThreads));
        pass_table_len += (size_t)b->max_slices[k];
        b->max_mx = std::max(b->max_mx, fft_len(nx));
        b->max_ny = std::max(b->max_ny, ny);
        b->max_my = std::max(b->max_my, fft_len(ny));
        I.g.nx = nx;
        I.g.ny = ny;
        I.g.x_min = gr.x_min;
        I.g.y_min = gr.y_min;
        I.g.inv_dx = 1.0 / gr.dx;
        I.g.inv_dy = 1.0 / gr.dy;
        const int slices = b->max_slices[k];
        BALLOC(I.dep.partial, sizeof(uint32_t) * (size_t)slices * ncell);
        BALLOC(I.dep.header, sizeof(BlockHeader) * (size_t)slices);
        BALLOC(I.dep.carry, sizeof(unsigned long long) * (size_t)ncell);
        I.dep.max_blocks = slices;
        I.nx = nx;
        I.ny = ny;
        I.mx = fft_len(nx);
        I.my = fft_len(ny);
        I.log2_mx = ilog2(I.mx);
        I.log2_my = ilog2(I.my);
        I.scale = n_k > 0 ? 1.0 / (kChargeOne * (double)n_k) : 0.0;
        const GridTables *gt = nullptr;
        for (const GridTables &t : tables)
            if (t.grid.nx == nx && t.grid.ny == ny && t.grid.dx == gr.dx && t.grid.dy == gr.dy)
                gt = &t;
        if (!gt) {
            GridTables t;
            t.grid = gr;
            BALLOC(t.stw_x, ce * I.mx);
            BALLOC(t.stw_y, ce * (2 * (size_t)I.my + 1));
            BALLOC(t.ghat_t, fe * (size_t)(I.my / 2 + 1) * I.mx);
            BALLOC(t.sx, fe * I.mx);
            BALLOC(t.sy, fe * (I.my / 2 + 1));
            st = b->mixed ? upload_grid_tables<float>(gr, t.ghat_t, t.stw_x, t.stw_y, t.sx, t.sy)
                          : upload_grid_tables<double>(gr, t.ghat_t, t.stw_x, t.stw_y, t.sx, t.sy);
            if (st) return st;
            tables.push_back(t);
            gt = &tables.back();
        }
        I.stw_x = gt->stw_x;
        I.stw_y = gt->stw_y;
        I.ghat_t = gt->ghat_t;
        I.sx = gt->sx;
        I.sy = gt->sy;
        BALLOC(I.spec_a, ce * (size_t)(I.my / 2 + 1) * nx);
        BALLOC(I.spec_bx, ce * (size_t)(I.my / 2 + 1) * nx);
        BALLOC(I.spec_by, ce * (size_t)(I.my / 2 + 1) * nx);
        BALLOC(I.ef, 2 * fe * ncell);
        SCPIC_HIP_TRY(hipMemset(I.dep.carry, 0, sizeof(unsigned long long) * ncell), "hipMemset");
        SCPIC_HIP_TRY(hipMemset(I.dep.header, 0xff, sizeof(BlockHeader) * slices), "hipMemset");
        SCPIC_HIP_TRY(hipMemset(I.ef, 0, 2 * fe * ncell), "hipMemset");
    }
    // Grid-phase workgroups in index order: the beams with the largest grids
    // and the most particles (more partial slices to sum) first, so that the
    // quick ones fill the end of each launch.
    std::vector<int> order(n_inst);
    for (int k = 0; k < n_inst; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int u, int v) {
        const int64_t cu = (int64_t)grids[u].nx * grids[u].ny, cv = (int64_t)grids[v].nx * grids[v].ny;
        if (cu != cv) return cu > cv;
        return offsets[u + 1] - offsets[u] > offsets[v + 1] - offsets[v];
    });
    for (int k : order) {
        BatchInstance &I = b->inst[k];
        I.row_block0 = b->total_rows;
        b->total_rows += I.nx;
        I.col_block0 = b->total_cols;
        b->total_cols += I.my / 2 + 1;
        for (int t = 0; t < I.nx; ++t) row_inst.push_back((uint16_t)k);
        for (int t = 0; t <= I.my / 2; ++t) col_inst.push_back((uint16_t)k);
    }
    BatchInstance *inst_dev;
    uint16_t *pass_dev, *row_dev, *col_dev;
    BALLOC(inst_dev, sizeof(BatchInstance) * n_inst);
    BALLOC(pass_dev, sizeof(uint16_t) * pass_table_len);
    BALLOC(row_dev, sizeof(uint16_t) * row_inst.size());
    BALLOC(col_dev, sizeof(uint16_t) * col_inst.size());
#undef BALLOC
    SCPIC_HIP_TRY(hipMemcpy(row_dev, row_inst.data(), sizeof(uint16_t) * row_inst.size(), hipMemcpyHostToDevice), "upload tables");
    SCPIC_HIP_TRY(hipMemcpy(col_dev, col_inst.data(), sizeof(uint16_t) * col_inst.size(), hipMemcpyHostToDevice), "upload tables");
    b->launch.inst = inst_dev;
    b->launch.pass_inst = pass_dev;
    b->launch.row_inst = row_dev;
    b->launch.col_inst = col_dev;
    b->launch.n_inst = n_inst;
    b->pass_table = pass_dev;
    SCPIC_HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if ((st = batch_layout(b, 1024, 1))) return st;
    SCPIC_HIP_TRY(prepare_pass_kernels(prop.sharedMemPerBlock), "hipFuncSetAttribute");
    SCPIC_HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    return SCPIC_OK;
}

bool same_shape(const std::vector<PassOp> &a, const std::vector<PassOp> &b)
{
    if (a.size() != b.size()) return false;
    for (size_t i = 0; i < a.size(); ++i)
        if (a[i].kick != b[i].kick || a[i].deposit != b[i].deposit) return false;
    return true;
}

// The cached schedule for per-beam op lists of one shape (ops[k] for beam k),
// its step table uploaded on first use.
scpic_status batch_schedule(scpic_batch *b, const std::vector<std::vector<PassOp>> &ops,
                            const scpic_particles *parts, BatchSchedule **out)
{
    const size_t n_ops = ops[0].size(), n = (size_t)b->n_inst;
    std::vector<BatchStep> table(n_ops * n);
    for (size_t j = 0; j < n_ops; ++j)
        for (size_t k = 0; k < n; ++k) {
            BatchStep &t = table[j * n + k];
            std::memset(&t, 0, sizeof(t));
            t.kappa = ops[k][j].kappa;
            t.els = ops[k][j].els;
        }
    std::vector<unsigned char> key;
    auto put = [&key](const void *d, size_t len) {
        const unsigned char *c = (const unsigned char *)d;
        key.insert(key.end(), c, c + len);
    };
    put(parts, sizeof(*parts));
    for (size_t j = 0; j < n_ops; ++j) {
        put(&ops[0][j].kick, sizeof(bool));
        put(&ops[0][j].deposit, sizeof(bool));
    }
    put(table.data(), sizeof(BatchStep) * table.size());
    for (auto &s : b->schedules)
        if (s.key == key) {
            s.last_use = ++b->use_counter;
            *out = &s;
            return SCPIC_OK;
        }
    if (b->schedules.size() >= kMaxSchedules) {
        // the evicted tables may still be read by queued work
        SCPIC_HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
        auto it = std::min_element(b->schedules.begin(), b->schedules.end(),
                                   [](const BatchSchedule &x, const BatchSchedule &y) {
                                       return x.last_use < y.last_use;
                                   });
        batch_drop_schedule(*it);
        b->schedules.erase(it);
    }
    BatchSchedule s;
    s.key = std::move(key);
    s.shape = ops[0];
    s.six.assign(n_ops, 0);
    for (size_t j = 0; j < n_ops; ++j)
        for (size_t k = 0; k < n; ++k)
            if (has_thick(ops[k][j].els)) s.six[j] = 1;
    hipError_t e = hipMalloc(&s.steps, sizeof(BatchStep) * std::max<size_t>(1, table.size()));
    if (e != hipSuccess) return fail(SCPIC_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    if (!table.empty()) {
        e = hipMemcpy(s.steps, table.data(), sizeof(BatchStep) * table.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            hipFree(s.steps);
            return fail_hip(e, "upload step table");
        }
    }
    s.last_use = ++b->use_counter;
    b->schedules.push_back(std::move(s));
    *out = &b->schedules.back();
    return SCPIC_OK;
}

scpic_status batch_enqueue(scpic_batch *b, hipStream_t s, const scpic_particles *parts,
                           const BatchSchedule &sch)
{
    const ParticlePtrs all = to_ptrs(parts);
    for (size_t j = 0; j < sch.shape.size(); ++j) {
        const PassOp &op = sch.shape[j];
        hipError_t e = launch_pass_batched(s, b->launch, all, sch.steps + j * b->n_inst, op.kick,
                                           b->mixed, op.deposit, sch.six[j] != 0,
                                           b->total_pass_blocks, b->pass_threads);
        if (e != hipSuccess) return fail_hip(e, "batched pass launch");
        if (op.deposit) {
            e = launch_solve_batched(s, b->launch, b->mixed, b->total_rows, b->total_cols,
                                     b->max_mx, b->max_ny, b->max_my, b->max_beam_blocks);
            if (e != hipSuccess) return fail_hip(e, "batched solve launch");
        }
    }
    return SCPIC_OK;
}

scpic_status batch_graph(scpic_batch *b, const scpic_particles *parts, BatchSchedule &sch)
{
    if (sch.exec) return SCPIC_OK;
    if (!b->capture_stream)
        SCPIC_HIP_TRY(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking), "hipStreamCreate");
    SCPIC_HIP_TRY(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal),
                  "hipStreamBeginCapture");
    scpic_status st = batch_enqueue(b, b->capture_stream, parts, sch);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(b->capture_stream, &graph);
    if (st) {
        if (graph) hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail_hip(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&sch.exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) {
        sch.exec = nullptr;
        return fail_hip(e, "hipGraphInstantiate");
    }
    return SCPIC_OK;
}

// Per-beam op lists of the first turn, a steady turn and the epilogue; they
// must share one shape (SCPIC_EUNSUPPORTED otherwise).
scpic_status batch_ops(scpic_batch *b, const scpic_particles *parts,
                       const scpic_element *const *turns, const int32_t *n_els,
                       std::vector<std::vector<PassOp>> &first,
                       std::vector<std::vector<PassOp>> &steady,
                       std::vector<std::vector<PassOp>> &tail, bool &any_sc0)
{
    for (int k = 0; k < b->n_inst; ++k) {
        std::vector<const scpic_element *> all, trailing;
        scpic_status st = collect_elements(turns[k], n_els[k], all, true);
        if (!st) st = check_longitudinal(all, parts);
        if (st) {
            g_last_error = "beam " + std::to_string(k) + ": " + g_last_error;
            return st;
        }
        bool any_sc = false;
        double last_kappa = 0.0;
        build_turn(all, true, first[k], any_sc, last_kappa, trailing);
        if (any_sc) {
            build_turn(all, false, steady[k], any_sc, last_kappa, trailing);
            emit_segment(tail[k], true, last_kappa, trailing, false);
        }
        if (k == 0) any_sc0 = any_sc;
        if (any_sc != any_sc0 || !same_shape(first[k], first[0]) ||
            !same_shape(steady[k], steady[0]) || !same_shape(tail[k], tail[0]))
            return fail(SCPIC_EUNSUPPORTED,
                        "beam " + std::to_string(k) +
                            ": its ring does not share the schedule of beam 0 (same number of "
                            "SC elements, at most 12 other elements between them)");
    }
    return SCPIC_OK;
}

void batch_drop_all_schedules(scpic_batch *b)
{
    for (auto &sc : b->schedules) batch_drop_schedule(sc);
    b->schedules.clear();
}

// Device scratch copy of the particles for timing runs (freed by the caller).
struct ScratchParts {
    scpic_particles p{};
    std::vector<void *> mem;
    ~ScratchParts()
    {
        for (void *m : mem) hipFree(m);
    }
};

scpic_status scratch_copy(hipStream_t s, const scpic_particles *src, ScratchParts &dst)
{
    dst.p = *src;
    const size_t n = (size_t)src->n;
    auto clone = [&](const void *from, size_t bytes, void **to) -> scpic_status {
        if (!from) {
            *to = nullptr;
            return SCPIC_OK;
        }
        hipError_t e = hipMalloc(to, bytes ? bytes : 1);
        if (e != hipSuccess) {
            *to = nullptr;
            return fail(SCPIC_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
        }
        dst.mem.push_back(*to);
        SCPIC_HIP_TRY(hipMemcpyAsync(*to, from, bytes, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
        return SCPIC_OK;
    };
    void *q;
    scpic_status st;
    if ((st = clone(src->x, 8 * n, &q))) return st;
    dst.p.x = (double *)q;
    if ((st = clone(src->px, 8 * n, &q))) return st;
    dst.p.px = (double *)q;
    if ((st = clone(src->y, 8 * n, &q))) return st;
    dst.p.y = (double *)q;
    if ((st = clone(src->py, 8 * n, &q))) return st;
    dst.p.py = (double *)q;
    if ((st = clone(src->sigma, 8 * n, &q))) return st;
    dst.p.sigma = (double *)q;
    if ((st = clone(src->psigma, 8 * n, &q))) return st;
    dst.p.psigma = (double *)q;
    if ((st = clone(src->w, 4 * n, &q))) return st;
    dst.p.w = (const float *)q;
    if ((st = clone(src->lost, n, &q))) return st;
    dst.p.lost = (uint8_t *)q;
    return SCPIC_OK;
}

}  // namespace

extern "C" {

scpic_status scpic_batch_autotune(scpic_batch *b, const scpic_particles *parts,
                                  const scpic_element *const *turns, const int32_t *n_els,
                                  int32_t trial_turns, int32_t *threads_out,
                                  int32_t *blocks_per_cu_out)
{
    g_last_error.clear();
    if (!b) return fail(SCPIC_EINVAL, "batch is NULL");
    if (scpic_status st = check_parts(parts)) return st;
    if (parts->n != b->offsets.back())
        return fail(SCPIC_EINVAL, "parts->n must equal offsets[n_inst] of the batch");
    if (!turns || !n_els) return fail(SCPIC_EINVAL, "turns and n_els must be non-NULL");
    if (trial_turns < 1 || trial_turns > 100)
        return fail(SCPIC_EINVAL, "trial_turns must be in [1, 100]");
    const int n = b->n_inst;
    std::vector<std::vector<PassOp>> first(n), steady(n), tail(n);
    bool any_sc = false;
    if (scpic_status st = batch_ops(b, parts, turns, n_els, first, steady, tail, any_sc)) return st;
    SCPIC_HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    batch_drop_all_schedules(b);
    ScratchParts scratch;
    if (scpic_status st = scratch_copy(b->stream, parts, scratch)) return st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    SCPIC_HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        hipEventDestroy(e0);
        return fail_hip(he, "hipEventCreate");
    }
    float best = -1.0f;
    int best_t = b->pass_threads, best_c = b->blocks_per_cu;
    scpic_status st = SCPIC_OK;
    const std::vector<std::vector<PassOp>> &timed = any_sc ? steady : first;
    for (int t : kTuneThreads) {
        for (int c : kTuneBlocksPerCu) {
            if ((st = batch_layout(b, t, c))) break;
            BatchSchedule *sch = nullptr;
            // one untimed turn (the first turn's schedule: it sets the
            // headers), then trial_turns timed steady turns
            if ((st = batch_schedule(b, first, &scratch.p, &sch))) break;
            if ((st = batch_enqueue(b, b->stream, &scratch.p, *sch))) break;
            if ((st = batch_schedule(b, timed, &scratch.p, &sch))) break;
            if ((he = hipEventRecord(e0, b->stream)) != hipSuccess) break;
            for (int r = 0; r < trial_turns && !st; ++r) st = batch_enqueue(b, b->stream, &scratch.p, *sch);
            if (st) break;
            if ((he = hipEventRecord(e1, b->stream)) != hipSuccess) break;
            if ((he = hipEventSynchronize(e1)) != hipSuccess) break;
            float ms = 0.0f;
            if ((he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
            if (best < 0.0f || ms < best) {
                best = ms;
                best_t = t;
                best_c = c;
            }
            batch_drop_all_schedules(b);
        }
        if (st || he != hipSuccess) break;
    }
    hipStreamSynchronize(b->stream);
    batch_drop_all_schedules(b);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st) return st;
    if (he != hipSuccess) return fail_hip(he, "timing the candidate shapes");
    if ((st = batch_layout(b, best_t, best_c))) return st;
    if (threads_out) *threads_out = best_t;
    if (blocks_per_cu_out) *blocks_per_cu_out = best_c;
    return SCPIC_OK;
}

scpic_status scpic_batch_create(scpic_batch **out, const scpic_grid *grids,
                                const int64_t *offsets, int32_t n_inst, int32_t precision,
                                void *hip_stream)
{
    g_last_error.clear();
    if (!out) return fail(SCPIC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!grids || !offsets) return fail(SCPIC_EINVAL, "grids and offsets must be non-NULL");
    if (n_inst < 1 || n_inst > 4096) return fail(SCPIC_EINVAL, "n_inst must be in [1, 4096]");
    if (precision != SCPIC_FP64 && precision != SCPIC_MIXED)
        return fail(SCPIC_EINVAL, "precision must be SCPIC_FP64 or SCPIC_MIXED");
    if (offsets[0] != 0) return fail(SCPIC_EINVAL, "offsets[0] must be 0");
    for (int k = 0; k < n_inst; ++k) {
        if (offsets[k + 1] < offsets[k])
            return fail(SCPIC_EINVAL, "offsets must not decrease (at beam " + std::to_string(k) + ")");
        if (scpic_status st = check_grid(&grids[k])) {
            g_last_error = "beam " + std::to_string(k) + ": " + g_last_error;
            return st;
        }
    }
    scpic_batch *b = new (std::nothrow) scpic_batch();
    if (!b) return fail(SCPIC_ENOMEM, "host allocation failed");
    scpic_status st = batch_create_impl(b, grids, offsets, n_inst, precision, hip_stream);
    if (st) {
        batch_free_all(b);
        delete b;
        return st;
    }
    *out = b;
    return SCPIC_OK;
}

scpic_status scpic_batch_destroy(scpic_batch *b)
{
    g_last_error.clear();
    if (!b) return SCPIC_OK;
    hipStreamSynchronize(b->stream);
    batch_free_all(b);
    delete b;
    return SCPIC_OK;
}

scpic_status scpic_batch_set_stream(scpic_batch *b, void *hip_stream)
{
    g_last_error.clear();
    if (!b) return fail(SCPIC_EINVAL, "batch is NULL");
    b->stream = (hipStream_t)hip_stream;
    return SCPIC_OK;
}

scpic_status scpic_track_batched(scpic_batch *b, const scpic_particles *parts,
                                 const scpic_element *const *turns, const int32_t *n_els,
                                 int32_t n_turns)
{
    g_last_error.clear();
    if (!b) return fail(SCPIC_EINVAL, "batch is NULL");
    if (scpic_status st = check_parts(parts)) return st;
    if (parts->n != b->offsets.back())
        return fail(SCPIC_EINVAL, "parts->n must equal offsets[n_inst] of the batch");
    if (!turns || !n_els) return fail(SCPIC_EINVAL, "turns and n_els must be non-NULL");
    if (n_turns < 0) return fail(SCPIC_EINVAL, "n_turns is negative");
    const int n = b->n_inst;
    std::vector<std::vector<PassOp>> first(n), steady(n), tail(n);
    bool any_sc0 = false;
    if (scpic_status st = batch_ops(b, parts, turns, n_els, first, steady, tail, any_sc0)) return st;
    if (n_turns == 0 || parts->n == 0) return SCPIC_OK;
    BatchSchedule *sch = nullptr;
    if (!any_sc0) {
        if (scpic_status st = batch_schedule(b, first, parts, &sch)) return st;
        for (int t = 0; t < n_turns; ++t)
            if (scpic_status st = batch_enqueue(b, b->stream, parts, *sch)) return st;
        return SCPIC_OK;
    }
    if (scpic_status st = batch_schedule(b, first, parts, &sch)) return st;
    if (scpic_status st = batch_enqueue(b, b->stream, parts, *sch)) return st;
    if (n_turns > 1) {
        if (scpic_status st = batch_schedule(b, steady, parts, &sch)) return st;
        if (scpic_status st = batch_graph(b, parts, *sch)) return st;
        for (int t = 1; t < n_turns; ++t)
            SCPIC_HIP_TRY(hipGraphLaunch(sch->exec, b->stream), "hipGraphLaunch");
    }
    if (scpic_status st = batch_schedule(b, tail, parts, &sch)) return st;
    return batch_enqueue(b, b->stream, parts, *sch);
}

scpic_status scpic_batch_get_field(scpic_batch *b, int32_t k, void *ex, void *ey)
{
    g_last_error.clear();
    if (!b) return fail(SCPIC_EINVAL, "batch is NULL");
    if (k < 0 || k >= b->n_inst) return fail(SCPIC_EINVAL, "beam index out of range");
    if (!ex || !ey) return fail(SCPIC_EINVAL, "ex and ey must be non-NULL");
    const BatchInstance &I = b->inst[k];
    hipError_t e = launch_interleave(b->stream, b->mixed, false, ex, ey, I.ef, I.nx * I.ny);
    if (e != hipSuccess) return fail_hip(e, "field copy launch");
    return SCPIC_OK;
}

}  // extern "C"

// ---- deposit without allocation ---------------------------------------------
//
// scpic_deposit_static runs the deposit of scpic_deposit (the same pass and
// reduction kernels) with its per-workgroup partials, headers and carry grid
// in one file-scope device array instead of a context's allocations.  The
// array's host-side name is not a device address: host code uses only the
// address hipGetSymbolAddress returns, looked up once per device.

namespace {

constexpr int kStaticBlocks = 64;  // workgroups of the allocation-free deposit
constexpr size_t kStaticHeaderBytes = sizeof(BlockHeader) * kStaticBlocks;
constexpr size_t kStaticCarryBytes = sizeof(unsigned long long) * kMaxCells;
constexpr size_t kStaticPartialBytes = sizeof(uint32_t) * (size_t)kStaticBlocks * kMaxCells;
constexpr size_t kStaticScratchBytes = kStaticHeaderBytes + kStaticCarryBytes + kStaticPartialBytes;
static_assert(kStaticScratchBytes == SCPIC_STATIC_SCRATCH_BYTES,
              "the header states the scratch size");
static_assert(kStaticHeaderBytes % 256 == 0 && kStaticCarryBytes % 256 == 0,
              "each part of the scratch starts 256-byte aligned");

__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_static_mutex;
unsigned char *g_static_ptr[kMaxDevices] = {};
bool g_static_ready[kMaxDevices] = {};

// Headers to "unknown" (every word -1: the first tile is the whole grid when
// it fits) and the carry grid's first ncell words to zero, by a kernel rather
// than a memset node, so that the call can be captured into a graph.
__global__ void __launch_bounds__(256)
    k_static_clear(BlockHeader *__restrict__ header, unsigned long long *__restrict__ carry,
                   int ncell)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < kStaticBlocks) {
        BlockHeader h;
        h.i0 = h.i1 = h.j0 = h.j1 = -1;
        h.count = -1;
        h.pad[0] = h.pad[1] = h.pad[2] = -1;
        header[t] = h;
    }
    if (t < ncell) carry[t] = 0ull;
}

// The scratch address on the current device and the pass kernels' LDS
// limits, set up once per device.
scpic_status static_scratch(unsigned char **out)
{
    int dev = 0;
    SCPIC_HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(SCPIC_EUNSUPPORTED, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_static_mutex);
    if (!g_static_ready[dev]) {
        void *ptr = nullptr;
        SCPIC_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
        hipDeviceProp_t prop;
        SCPIC_HIP_TRY(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
        SCPIC_HIP_TRY(prepare_pass_kernels(prop.sharedMemPerBlock), "hipFuncSetAttribute");
        g_static_ptr[dev] = (unsigned char *)ptr;
        g_static_ready[dev] = true;
    }
    *out = g_static_ptr[dev];
    return SCPIC_OK;
}

}  // namespace

extern "C" {

scpic_status scpic_deposit_static(const scpic_grid *grid, const scpic_particles *parts,
                                  int64_t *rho, int64_t *n_in, void *hip_stream)
{
    g_last_error.clear();
    if (!grid) return fail(SCPIC_EINVAL, "grid is NULL");
    if (scpic_status st = check_grid(grid)) return st;
    if (scpic_status st = check_parts(parts)) return st;
    if (!rho) return fail(SCPIC_EINVAL, "rho is NULL");
    // a workgroup's header counts its particles in 32 bits
    if (parts->n > (int64_t)kStaticBlocks * INT32_MAX)
        return fail(SCPIC_EUNSUPPORTED, "at most 64 * (2^31 - 1) particles per call");
    unsigned char *base = nullptr;
    if (scpic_status st = static_scratch(&base)) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    DepositTarget dep;
    dep.header = (BlockHeader *)base;
    dep.carry = (unsigned long long *)(base + kStaticHeaderBytes);
    dep.partial = (uint32_t *)(base + kStaticHeaderBytes + kStaticCarryBytes);
    dep.max_blocks = kStaticBlocks;
    const int ncell = grid->nx * grid->ny;
    hipLaunchKernelGGL(k_static_clear, dim3((std::max(ncell, kStaticBlocks) + 255) / 256),
                       dim3(256), 0, s, dep.header, dep.carry, ncell);
    SCPIC_HIP_TRY(hipGetLastError(), "scratch clear launch");
    GridGeom g;
    g.nx = grid->nx;
    g.ny = grid->ny;
    g.x_min = grid->x_min;
    g.y_min = grid->y_min;
    g.inv_dx = 1.0 / grid->dx;
    g.inv_dy = 1.0 / grid->dy;
    constexpr int kThreads = 1024;
    const int blocks =
        parts->n > 0 ? (int)std::min<int64_t>(kStaticBlocks, (parts->n + kThreads - 1) / kThreads)
                     : 0;
    PassElements none;
    std::memset(&none, 0, sizeof(none));
    if (blocks > 0) {
        ParticlePtrs p = to_ptrs(parts);
        p.stream = false;
        SCPIC_HIP_TRY(launch_pass(s, p, g, false, false, nullptr, 0.0, none, true, dep, blocks,
                                  kThreads),
                      "deposit pass launch");
    }
    SCPIC_HIP_TRY(launch_reduce(s, dep, blocks, grid->nx, grid->ny, rho, n_in), "reduce launch");
    return SCPIC_OK;
}

}  // extern "C"
