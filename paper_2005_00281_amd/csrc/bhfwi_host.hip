// bhfwi_host.hip -- C-ABI of libbhfwi: validation, layout planning, PML
// profiles and the launch sequences of the forward, adjoint and update steps.
#include "bhfwi.h"
#include "bhfwi_kernels.hip"
#include "bhfwi_tb_fwd.hip"
#include "bhfwi_tb_adj.hip"
#include "bhfwi_o4.hip"
#include "bhfwi_o4_tb.hip"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using bhfwi::ShotDev;

namespace {

constexpr int kPartBlocks = 1024;  // blocks of the two-level reductions
constexpr int64_t kAlign = 64;     // floats (256 bytes) between packed blocks

int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Packed lengths (floats) of one shot: its cells, forward state (6 fields and
// 4 PML memories per strip) and adjoint state (6 fields and 5 per strip).
struct ShotLens {
    int64_t cells, fst, ast;
};

ShotLens shot_lens(const bhfwi_shot& h)
{
    const int64_t NR = (int64_t)h.nr + h.npml_r, NZ = (int64_t)h.nz + 2 * (int64_t)h.npml_z;
    const int64_t pr = (int64_t)h.npml_r * NZ, pz = NR * 2 * h.npml_z;
    return {align_up(NR * NZ), align_up(6 * NR * NZ + 4 * pr + 4 * pz),
            align_up(6 * NR * NZ + 5 * pr + 5 * pz)};
}

bhfwi_plan_bytes_t group_bytes(const bhfwi_shot* shots, const int* idx, int n, int K)
{
    int64_t C = 0, F = 0, A = 0;
    int ntmax = 0;
    for (int q = 0; q < n; ++q) {
        const ShotLens l = shot_lens(shots[idx[q]]);
        C += l.cells;
        F += l.fst;
        A += l.ast;
        ntmax = std::max(ntmax, shots[idx[q]].nt);
    }
    const int64_t nseg = (ntmax + K - 1) / K;
    bhfwi_plan_bytes_t b{};
    b.ckpt_every = K;
    b.fwd_ws_bytes = 8 * F;
    b.ckpt_bytes = 4 * std::max<int64_t>(0, nseg - 1) * F;
    b.adj_ws_bytes = 4 * (2 * A + 2 * (int64_t)K * C);
    b.acc_bytes = 16 * C;
    b.total_bytes = b.fwd_ws_bytes + b.ckpt_bytes + b.adj_ws_bytes + b.acc_bytes;
    return b;
}

int best_interval(const bhfwi_shot* shots, const int* idx, int n)
{
    int64_t C = 0, F = 0;
    int ntmax = 0;
    for (int q = 0; q < n; ++q) {
        const ShotLens l = shot_lens(shots[idx[q]]);
        C += l.cells;
        F += l.fst;
        ntmax = std::max(ntmax, shots[idx[q]].nt);
    }
    const int64_t k = (int64_t)std::sqrt((double)ntmax * (double)F / (2.0 * (double)C));
    int best = 0;
    int64_t best_b = 0;
    for (int64_t cand : {k / 8 * 8, (k + 7) / 8 * 8}) {
        const int K = (int)std::min<int64_t>(std::max<int64_t>(8, cand), ntmax);
        const int64_t b = group_bytes(shots, idx, n, K).total_bytes;
        if (!best || b < best_b) {
            best = K;
            best_b = b;
        }
    }
    return best;
}

// message of the last failed context-free call on this thread (bhfwi_create,
// bhfwi_misfit_noalloc), readable through bhfwi_last_error(NULL)
thread_local std::string g_create_err;

}  // namespace

// Device scratch of the allocation-free misfit (bhfwi_misfit_noalloc): the
// partial sums of its two-level reduction, one per block of the first pass,
// whatever the number of samples.  Each GPU the library runs on holds its
// own copy (8 KiB) until the process ends; calls on one GPU share it.
constexpr int kScratchParts = 1024;
static __device__ __align__(256) double scratch[kScratchParts];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};  // device address of `scratch`, per device

// Device address of `scratch` on device dev, looked up once per device with
// that device current (the array's name in host code is only a host-side
// stand-in and must never reach a kernel).
int scratch_address(int dev, double** out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
        void* p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) {
            g_create_err = std::string("misfit_noalloc: hipGetSymbolAddress(scratch): ") +
                           hipGetErrorString(e);
            return BHFWI_EHIP;
        }
        g_scratch_dev[dev] = (double*)p;
    }
    *out = g_scratch_dev[dev];
    return BHFWI_OK;
}

}  // namespace

// A temporally blocked kernel shape: T steps per launch, TRE tile rows
// including the halo, W waves per workgroup; T = 0 means one step per launch.
struct Shape {
    int T, TRE, W;
};

// Tiles (shot, k0, i0, first radial row written back) of one temporally
// blocked shape in two lists:
// [0] tiles clear of every PML layer, run by the PML-free kernel of the shape;
// [1] the tiles that touch a PML layer, cut into sub-tiles of shape `pml`
// (same T, fewer rows) and run by the kernel that carries the PML memories.
// Each list is ordered by the nt of its shot (non-increasing).
struct TileSet {
    std::vector<int4> t[2];
    std::vector<int> nt[2];
    int4* d[2] = {nullptr, nullptr};
    Shape pml{0, 0, 0};
};

struct bhfwi_ctx {
    int device = 0;
    int nshot = 0;
    int64_t model_len = 0;
    int ckpt_every = 0;
    std::vector<bhfwi_shot> shots;
    std::vector<int32_t> rec;
    std::vector<ShotDev> sd;
    int64_t cells = 0, fst_len = 0, ast_len = 0, trace_len = 0, wave_len = 0, cell_steps = 0;
    int nt_max = 0, nseg = 0;
    int order = 2;  // spatial order of the step: 2 or 4 (bhfwi_set_order)
    int* d_tile4 = nullptr;  // fourth order: first tile of each shot (nshot + 1)
    int ntile4 = 0;
    Shape f4{2, 32, 16};  // fourth-order forward time blocks (T = 0: one step per launch)
    TileSet f4tiles;      // their tiles (halo 3T)
    bhfwi_tune tune{};
    std::vector<int4> work;
    std::vector<int> work_nt;  // nt of each work item's shot, non-increasing
    TileSet ftiles, atiles;    // temporally blocked tiles of the forward / adjoint shape
    TileSet xtiles;            // the adjoint's with extra outputs, when they differ
    ShotDev* d_shots = nullptr;
    int* d_rec = nullptr;
    float* d_pml_r = nullptr;
    float* d_pml_z = nullptr;
    int4* d_work = nullptr;
    void* d_scratch = nullptr;
    int* d_status = nullptr;  // device word raised by kernels that see non-finite sums
    float* wgrad = nullptr;       // wavelet gradient output of the adjoint being recorded
    hipStream_t cap_stream = nullptr;  // private stream that graphs are captured on
    hipStream_t pml_stream = nullptr;  // second stream for the PML tiles of a block
    hipStream_t rec_stream = nullptr;  // recompute stream of the overlapped adjoint
    hipEvent_t ev_rec_start = nullptr, ev_rec[2] = {nullptr, nullptr},
               ev_adj[2] = {nullptr, nullptr};
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    struct Graph {
        std::vector<uintptr_t> key;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;  // small cache, most recent last
    // per-launch event pairs of the instrumented mode: kind 0 fwd, 1 rec, 2 adj
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, int>> ev_used;  // (kind, index of the start event)
    std::string err;
};

namespace {

int fail(bhfwi_ctx* c, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPOK(ctx, call)                                                              \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail((ctx), BHFWI_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

int grid1d(int64_t n, int cap = 4096)
{
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    return (int)std::min<int64_t>(g, cap);
}

// Complex-frequency-shifted PML (reading of the paper's PML citation):
// penetration x in (0, 1], d = d0 x^2, alpha = pi f0 (1 - x), kappa = 1,
// b = exp(-(d + alpha) dt), a = d (b - 1) / (d + alpha); a = 0, b = 1 outside.
void pml_coef(double x, double d0, double f0, double dt, float* a, float* b)
{
    if (!(x > 0.0)) {
        *a = 0.0f;
        *b = 1.0f;
        return;
    }
    const double d = d0 * x * x;
    const double al = M_PI * f0 * (1.0 - x);
    const double bb = std::exp(-(d + al) * dt);
    *b = (float)bb;
    *a = (float)(d * (bb - 1.0) / (d + al));
}

Shape pml_shape(Shape sh, bool adj);

Shape fwd_shape(const bhfwi_ctx* c)
{
    const bhfwi_tune& t = c->tune;
    return t.tb_steps >= 2 ? Shape{t.tb_steps, t.tb_rows, t.tb_waves} : Shape{0, 0, 0};
}

// The adjoint runs its own shape when adj_tb_steps >= 2, one step per launch
// when it is 1, and the forward's shape when it is 0.
Shape adj_shape(const bhfwi_ctx* c)
{
    const bhfwi_tune& t = c->tune;
    if (t.adj_tb_steps >= 2) return Shape{t.adj_tb_steps, t.adj_tb_rows, t.adj_tb_waves};
    if (t.adj_tb_steps == 1) return Shape{0, 0, 0};
    return fwd_shape(c);
}

bool adj_int_ok(Shape sh);

// The adjoint shape of the launches with extra outputs (density correlation,
// pseudo-Hessian): an interior shape with four rows per thread holds its
// state in 128 VGPRs only by reading values back from LDS, and the four extra
// register sums per row would spill, so those launches take the shape with
// three rows per thread and the same T and waves; T = 0 when they run the
// adjoint shape itself.
Shape adj_x_shape(const bhfwi_ctx* c)
{
    const Shape a = adj_shape(c);
    if (a.T >= 2 && a.TRE >= 4 * a.W) {
        const Shape f{a.T, 3 * a.W, a.W};
        if (adj_int_ok(f)) return f;
    }
    return Shape{0, 0, 0};
}

// Whether a tile of shape sh at (i0, k0) -- with its halo -- reaches a PML
// layer: the test the kernels apply to pick their PML loop.
bool touches_pml(const ShotDev& S, Shape sh, int i0, int k0)
{
    const int ihi = i0 - sh.T + sh.TRE - 1, klo = k0 - sh.T, khi = k0 - sh.T + 63;
    return ihi >= S.nr || klo < S.pz || khi >= S.NZ - S.pz;
}

void build_tiles(const bhfwi_ctx* c, const std::vector<int>& order, Shape sh, Shape pml,
                 TileSet* ts, bool overlap = false)
{
    for (int q = 0; q < 2; ++q) {
        ts->t[q].clear();
        ts->nt[q].clear();
    }
    ts->pml = pml;
    if (sh.T < 2) return;
    // Columns of TZ axial rows (the same T, hence TZ, for both shapes).  In a
    // column clear of the axial PML, interior tiles of TR rows cover the rows
    // whose haloed window stays below the radial PML; the rest of the
    // column, and every column that reaches the axial PML, is covered by PML
    // tiles of TRp rows.  With overlap (tune fwd_tile_overlap, the forward
    // only) one more interior tile ends where the radial layer's halo begins;
    // its window overlaps the interior tile below it, but it writes back only
    // the rows above that tile, so every cell keeps one writer, and the PML
    // tiles then cover only the rows that need them.  A tile is (shot, first
    // axial row, first owned radial row, first radial row it writes).
    const int TR = sh.TRE - 2 * sh.T, TZ = 64 - 2 * sh.T, TRp = pml.TRE - 2 * pml.T;
    std::vector<int4> tl[2];  // (k0, i0, first written row, 0) of one shot's tiles
    for (int s : order) {
        const ShotDev& S = c->sd[s];
        tl[0].clear();
        tl[1].clear();
        for (int k0 = 0; k0 < S.NZ; k0 += TZ) {
            int i0 = 0;
            if (!touches_pml(S, sh, 0, k0)) {
                for (; i0 < S.NR && !touches_pml(S, sh, i0, k0); i0 += TR)
                    tl[0].push_back(make_int4(k0, i0, i0, 0));
                const int last = S.nr - (sh.TRE - sh.T);  // highest start clear of the layer
                if (overlap && i0 < S.NR && last > i0 - TR && last < i0 &&
                    !touches_pml(S, sh, last, k0)) {
                    tl[0].push_back(make_int4(k0, last, i0, 0));
                    i0 = last + TR;
                }
            }
            for (; i0 < S.NR; i0 += TRp) tl[1].push_back(make_int4(k0, i0, i0, 0));
        }
        for (int q = 0; q < 2; ++q) {
            if (c->tune.tile_map == 0)  // axial tile fastest
                std::stable_sort(tl[q].begin(), tl[q].end(), [](int4 a, int4 b) {
                    return a.y != b.y ? a.y < b.y : a.x < b.x;
                });
            for (const int4 kt : tl[q]) {
                ts->t[q].push_back(make_int4(s, kt.x, kt.y, kt.z));
                ts->nt[q].push_back(S.nt);
            }
        }
    }
}

int upload_tiles(bhfwi_ctx* c, TileSet* ts)
{
    for (int q = 0; q < 2; ++q) {
        if (ts->d[q]) {
            HIPOK(c, hipFree(ts->d[q]));
            ts->d[q] = nullptr;
        }
        if (!ts->t[q].empty()) {
            HIPOK(c, hipMalloc(&ts->d[q], sizeof(int4) * ts->t[q].size()));
            HIPOK(c, hipMemcpy(ts->d[q], ts->t[q].data(), sizeof(int4) * ts->t[q].size(),
                               hipMemcpyHostToDevice));
        }
    }
    return BHFWI_OK;
}

void rebuild_work(bhfwi_ctx* c)
{
    c->work.clear();
    c->work_nt.clear();
    std::vector<int> order(c->nshot);
    for (int s = 0; s < c->nshot; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return c->sd[a].nt > c->sd[b].nt; });
    const int R = std::max(1, c->tune.rows_per_wave);
    for (int s : order) {
        const ShotDev& S = c->sd[s];
        const int strips = (S.NZ + bhfwi::kOwn - 1) / bhfwi::kOwn;
        for (int i0 = 0; i0 < S.NR; i0 += R)
            for (int j = 0; j < strips; ++j) {
                c->work.push_back(make_int4(s, j * bhfwi::kOwn, i0, std::min(i0 + R, S.NR)));
                c->work_nt.push_back(S.nt);
            }
    }
    const Shape fs = fwd_shape(c), as = adj_shape(c), xs = adj_x_shape(c);
    build_tiles(c, order, fs, pml_shape(fs, false), &c->ftiles, c->tune.fwd_tile_overlap != 0);
    build_tiles(c, order, as, pml_shape(as, true), &c->atiles);
    build_tiles(c, order, xs, pml_shape(xs, true), &c->xtiles);
    // fourth-order forward blocks: a three-cell halo per step, one shape for
    // the interior and the PML tiles
    const Shape h4{3 * c->f4.T, c->f4.TRE, c->f4.W};
    build_tiles(c, order, h4, h4, &c->f4tiles);
}

int upload_work(bhfwi_ctx* c)
{
    if (c->d_work) {
        HIPOK(c, hipFree(c->d_work));
        c->d_work = nullptr;
    }
    HIPOK(c, hipMalloc(&c->d_work, sizeof(int4) * c->work.size()));
    HIPOK(c, hipMemcpy(c->d_work, c->work.data(), sizeof(int4) * c->work.size(),
                       hipMemcpyHostToDevice));
    if (int rc = upload_tiles(c, &c->ftiles)) return rc;
    if (int rc = upload_tiles(c, &c->atiles)) return rc;
    if (int rc = upload_tiles(c, &c->f4tiles)) return rc;
    return upload_tiles(c, &c->xtiles);
}

int default_rows(const bhfwi_ctx* c)
{
    // aim for >= 8192 waves per step (32 per CU) before lengthening the march
    int64_t strip_rows = 0;
    for (const ShotDev& S : c->sd)
        strip_rows += (int64_t)((S.NZ + bhfwi::kOwn - 1) / bhfwi::kOwn) * S.NR;
    int64_t r = strip_rows / 8192;
    return (int)std::max<int64_t>(4, std::min<int64_t>(64, r));
}

int active_items(const bhfwi_ctx* c, int n)
{
    // work_nt is non-increasing: count items whose shot still runs at step n
    auto it = std::partition_point(c->work_nt.begin(), c->work_nt.end(),
                                   [n](int nt) { return nt > n; });
    return (int)(it - c->work_nt.begin());
}

int active_tiles(const TileSet& ts, int q, int n)
{
    auto it = std::partition_point(ts.nt[q].begin(), ts.nt[q].end(),
                                   [n](int nt) { return nt > n; });
    return (int)(it - ts.nt[q].begin());
}

int check_ctx(bhfwi_ctx* c)
{
    if (!c) return BHFWI_EINVAL;
    HIPOK(c, hipSetDevice(c->device));
    return BHFWI_OK;
}

void launch_fill(hipStream_t st, float* p, int64_t n, float v)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(bhfwi::k_fill, dim3(grid1d(n)), dim3(256), 0, st, p, (long long)n, v);
}

// Chunks of up to 4 rows use the kernels that issue every load up front.
#define BHFWI_DISPATCH(R, KER, ...)                                                         \
    do {                                                                                    \
        switch (R) {                                                                        \
        case 1: hipLaunchKernelGGL(KER<1>, __VA_ARGS__); break;                             \
        case 2: hipLaunchKernelGGL(KER<2>, __VA_ARGS__); break;                             \
        case 3: hipLaunchKernelGGL(KER<3>, __VA_ARGS__); break;                             \
        case 4: hipLaunchKernelGGL(KER<4>, __VA_ARGS__); break;                             \
        default: hipLaunchKernelGGL(KER<0>, __VA_ARGS__); break;                            \
        }                                                                                   \
    } while (0)

// Instrumented mode: an event pair around one launch (events are pooled).
struct EvScope {
    bhfwi_ctx* c;
    hipStream_t st;
    int idx = -1;
    EvScope(bhfwi_ctx* c_, hipStream_t st_, int kind) : c(c_), st(st_)
    {
        if (!c->tune.time_kernels || c->tune.use_graph) return;
        idx = (int)(2 * c->ev_used.size());
        while ((int)c->ev_pool.size() < idx + 2) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) {
                idx = -1;
                return;
            }
            c->ev_pool.push_back(e);
        }
        c->ev_used.push_back({kind, idx});
        (void)hipEventRecord(c->ev_pool[idx], st);
    }
    ~EvScope()
    {
        if (idx >= 0) (void)hipEventRecord(c->ev_pool[idx + 1], st);
    }
};

void fwd_launch(bhfwi_ctx* c, hipStream_t st, int n, const float* lam, const float* mu,
                const float* rho, const float* wav, const float* in, float* out, float* traces,
                float* hist)
{
    const int nact = active_items(c, n);
    if (nact <= 0) return;
    const int wpb = c->tune.waves_per_block;
    EvScope ev(c, st, hist ? 1 : 0);
    BHFWI_DISPATCH(c->tune.rows_per_wave, bhfwi::k_fwd_step, dim3((nact + wpb - 1) / wpb),
                   dim3(64 * wpb), 0, st, c->d_shots, c->d_work, nact, n, lam, mu, rho, wav,
                   c->d_rec, c->d_pml_r, c->d_pml_z, in, out, traces, hist, (long long)c->cells);
}

void adj_launch(bhfwi_ctx* c, hipStream_t st, int n, const float* lam, const float* mu,
                const float* rho, const float* resid, const float* in, float* out,
                const float* hist, float* acc, float* acc_rho, float* acc_h)
{
    const int nact = active_items(c, n);
    if (nact <= 0) return;
    const int wpb = c->tune.waves_per_block;
    EvScope ev(c, st, 2);
    BHFWI_DISPATCH(c->tune.rows_per_wave, bhfwi::k_adj_step, dim3((nact + wpb - 1) / wpb),
                   dim3(64 * wpb), 0, st, c->d_shots, c->d_work, nact, n, lam, mu, rho, c->d_rec,
                   resid, c->d_pml_r, c->d_pml_z, in, out, hist, acc, acc_rho, acc_h,
                   c->wgrad, (long long)c->cells);
}

// Fourth-order step n in one launch (tiles of TK x TI cells).
void fwd4_launch(bhfwi_ctx* c, hipStream_t st, int n, const float* lam, const float* mu,
                 const float* rho, const float* wav, const float* in, float* out, float* traces,
                 float* hist)
{
    EvScope ev(c, st, hist ? 1 : 0);
    hipLaunchKernelGGL(bhfwi::o4::k_fwd4, dim3((unsigned)c->ntile4),
                       dim3(bhfwi::o4::TK * bhfwi::o4::TI), 0, st, c->d_shots, c->d_tile4,
                       c->nshot, n, lam, mu, rho, wav, c->d_rec, c->d_pml_r, c->d_pml_z, in, out,
                       traces, hist, (long long)c->cells);
}

// Fourth-order forward steps n0 .. n0 + nsteps - 1 in time blocks (interior
// tiles, then PML tiles; the shapes compiled are listed in BHFWI_F4).
#define BHFWI_F4(X) X(2, 32, 16)
void fwd4_tb_launch(bhfwi_ctx* c, hipStream_t st, int n0, int nsteps, const float* lam,
                    const float* mu, const float* rho, const float* wav, const float* in,
                    float* out, float* traces, float* hist)
{
    const TileSet& ts = c->f4tiles;
    const int na[2] = {active_tiles(ts, 0, n0), active_tiles(ts, 1, n0)};
    if (na[0] + na[1] <= 0) return;
    EvScope ev(c, st, hist ? 1 : 0);
    for (int q = 0; q < 2; ++q) {
        const int nact = na[q];
        if (nact <= 0) continue;
        const int T = c->f4.T, TRE = c->f4.TRE, W = c->f4.W;
#define BHFWI_F4L(TT, RR, WW)                                                                  \
        if (T == TT && TRE == RR && W == WW) {                                                 \
            if (q == 0)                                                                        \
                hipLaunchKernelGGL((bhfwi::o4::k_fwd4_tb<TT, RR, WW, 0>), dim3(nact),          \
                                   dim3(64 * WW), 0, st, c->d_shots, ts.d[q], nact,            \
                                   c->tune.tile_map, n0, nsteps, lam, mu, rho, wav, c->d_rec,  \
                                   c->d_pml_r, c->d_pml_z, in, out, traces, hist,              \
                                   (long long)(2 * c->cells), (long long)c->cells);            \
            else                                                                               \
                hipLaunchKernelGGL((bhfwi::o4::k_fwd4_tb<TT, RR, WW, 1>), dim3(nact),          \
                                   dim3(64 * WW), 0, st, c->d_shots, ts.d[q], nact,            \
                                   c->tune.tile_map, n0, nsteps, lam, mu, rho, wav, c->d_rec,  \
                                   c->d_pml_r, c->d_pml_z, in, out, traces, hist,              \
                                   (long long)(2 * c->cells), (long long)c->cells);            \
            continue;                                                                          \
        }
        BHFWI_F4(BHFWI_F4L)
#undef BHFWI_F4L
    }
}

// Fourth-order adjoint steps n_hi, n_hi - 1, ... (nsteps of them) in one time
// block with the correlation; acc_rho and acc_h (nullable) select the
// density correlation and the pseudo-Hessian as in adj4_launch.
void adj4_tb_launch(bhfwi_ctx* c, hipStream_t st, int n_hi, int nsteps, const float* lam,
                    const float* mu, const float* rho, const float* resid, const float* in,
                    float* out, const float* hist_hi, float* acc, float* acc_rho, float* acc_h)
{
    const int xm = (acc_rho ? 1 : 0) | (acc_h ? 2 : 0);
    const TileSet& ts = c->f4tiles;
    const int n_lo = n_hi - nsteps + 1;
    const int na[2] = {active_tiles(ts, 0, n_lo), active_tiles(ts, 1, n_lo)};
    if (na[0] + na[1] <= 0) return;
    EvScope ev(c, st, 2);
    for (int q = 0; q < 2; ++q) {
        const int nact = na[q];
        if (nact <= 0) continue;
        const int T = c->f4.T, TRE = c->f4.TRE, W = c->f4.W;
#define BHFWI_A4K(TT, RR, WW, PP, XX)                                                          \
    hipLaunchKernelGGL((bhfwi::o4::k_adj4_tb<TT, RR, WW, PP, XX>), dim3(nact), dim3(64 * WW),    \
                       0, st, c->d_shots, ts.d[q], nact, c->tune.tile_map, n_hi, nsteps, lam,   \
                       mu, rho, c->d_rec, resid, c->d_pml_r, c->d_pml_z, in, out, hist_hi,      \
                       (long long)(2 * c->cells), acc, acc_rho, acc_h, (long long)c->cells)
#define BHFWI_A4L(TT, RR, WW)                                                                  \
        if (T == TT && TRE == RR && W == WW) {                                                 \
            if (q == 0) {                                                                      \
                switch (xm) {                                                                  \
                case 1: BHFWI_A4K(TT, RR, WW, 0, 1); break;                                    \
                case 2: BHFWI_A4K(TT, RR, WW, 0, 2); break;                                    \
                case 3: BHFWI_A4K(TT, RR, WW, 0, 3); break;                                    \
                default: BHFWI_A4K(TT, RR, WW, 0, 0); break;                                   \
                }                                                                              \
            } else {                                                                           \
                switch (xm) {                                                                  \
                case 1: BHFWI_A4K(TT, RR, WW, 1, 1); break;                                    \
                case 2: BHFWI_A4K(TT, RR, WW, 1, 2); break;                                    \
                case 3: BHFWI_A4K(TT, RR, WW, 1, 3); break;                                    \
                default: BHFWI_A4K(TT, RR, WW, 1, 0); break;                                   \
                }                                                                              \
            }                                                                                  \
            continue;                                                                          \
        }
        BHFWI_F4(BHFWI_A4L)
#undef BHFWI_A4L
#undef BHFWI_A4K
    }
}

bool f4_ok(Shape sh)
{
#define BHFWI_F4S(TT, RR, WW) \
    if (sh.T == TT && sh.TRE == RR && sh.W == WW) return true;
    BHFWI_F4(BHFWI_F4S)
#undef BHFWI_F4S
    return sh.T == 0;
}

// Fourth-order adjoint step n fused with the correlation, in one launch;
// acc_rho and acc_h (nullable) select the kernels that also accumulate the
// density correlation and the pseudo-Hessian.
void adj4_launch(bhfwi_ctx* c, hipStream_t st, int n, const float* lam, const float* mu,
                 const float* rho, const float* resid, const float* in, float* out,
                 const float* hist, float* acc, float* acc_rho, float* acc_h)
{
    EvScope ev(c, st, 2);
    const int xm = (acc_rho ? 1 : 0) | (acc_h ? 2 : 0);
#define BHFWI_A4(XX)                                                                          \
    hipLaunchKernelGGL(bhfwi::o4::k_adj4<XX>, dim3((unsigned)c->ntile4),                     \
                       dim3(bhfwi::o4::TK * bhfwi::o4::TI), 0, st, c->d_shots, c->d_tile4,   \
                       c->nshot, n, lam, mu, rho, c->d_rec, resid, c->d_pml_r, c->d_pml_z, in, \
                       out, hist, acc, acc_rho, acc_h, (long long)c->cells)
    switch (xm) {
    case 0: BHFWI_A4(0); break;
    case 1: BHFWI_A4(1); break;
    case 2: BHFWI_A4(2); break;
    default: BHFWI_A4(3); break;
    }
#undef BHFWI_A4
}

// Supported temporally blocked shapes: (steps T, tile rows incl. halo,
// waves).  *_PML lists the shapes whose kernel carries the PML memories (all
// tiles may use them); *_INT adds shapes compiled only without them, for
// tiles clear of the PML: with fewer live values per cell they afford more
// rows per thread.  A tile of an interior-only shape that touches a PML layer
// is cut into sub-tiles of a *_PML shape with the same T (pml_shape).
#define BHFWI_ADJ_PML(X) \
    X(2, 16, 4) X(3, 16, 4) X(4, 16, 4) X(2, 16, 8) X(3, 16, 8) X(4, 16, 8) X(2, 24, 8) \
    X(3, 24, 8) X(4, 24, 8) X(6, 24, 8) X(4, 32, 8) X(6, 32, 8) X(8, 32, 8) X(2, 16, 16) \
    X(3, 16, 16) X(4, 16, 16) X(4, 32, 16) X(6, 32, 16) X(8, 32, 16)
#define BHFWI_ADJ_INT(X) \
    BHFWI_ADJ_PML(X) X(4, 48, 16) X(6, 48, 16) X(8, 48, 16) X(8, 64, 16)
#define BHFWI_FWD_PML(X) BHFWI_ADJ_PML(X) X(4, 48, 16) X(6, 48, 16) X(8, 48, 16)
#define BHFWI_FWD_INT(X) BHFWI_FWD_PML(X) X(4, 64, 16) X(8, 64, 16)

#define BHFWI_TBS(TT, RR, WW) \
    if (sh.T == TT && sh.TRE == RR && sh.W == WW) return true;
bool fwd_pml_ok(Shape sh) { BHFWI_FWD_PML(BHFWI_TBS) return false; }
bool fwd_int_ok(Shape sh) { BHFWI_FWD_INT(BHFWI_TBS) return false; }
bool adj_pml_ok(Shape sh) { BHFWI_ADJ_PML(BHFWI_TBS) return false; }
bool adj_int_ok(Shape sh) { BHFWI_ADJ_INT(BHFWI_TBS) return false; }
#undef BHFWI_TBS

// Shape for the PML tiles of interior shape sh: sh itself when its kernel can
// carry the PML, else the PML-capable shape with the same T whose owned rows
// divide sh's (most rows, then most waves); T = 0 if there is none.  (Taller
// PML tiles were measured slower: the PML band of a single shot then holds
// fewer workgroups than the GPU has compute units.)
Shape pml_shape(Shape sh, bool adj)
{
    if (sh.T < 2) return Shape{0, 0, 0};
    if (adj ? adj_pml_ok(sh) : fwd_pml_ok(sh)) return sh;
    Shape best{0, 0, 0};
    const int TR = sh.TRE - 2 * sh.T;
    auto consider = [&](int T, int R, int W) {
        const int TRp = R - 2 * T;
        if (T != sh.T || TRp <= 0 || TR % TRp) return;
        if (R > best.TRE || (R == best.TRE && W > best.W)) best = Shape{T, R, W};
    };
#define BHFWI_TBP(TT, RR, WW) consider(TT, RR, WW);
    if (adj) {
        BHFWI_ADJ_PML(BHFWI_TBP)
    } else {
        BHFWI_FWD_PML(BHFWI_TBP)
    }
#undef BHFWI_TBP
    return best;
}

bool fwd_supported(int T, int TRE, int W)
{
    const Shape sh{T, TRE, W};
    return fwd_int_ok(sh) && pml_shape(sh, false).T >= 2;
}
bool adj_supported(int T, int TRE, int W)
{
    const Shape sh{T, TRE, W};
    return adj_int_ok(sh) && pml_shape(sh, true).T >= 2;
}

// The PML tiles of a block run on a second stream, forked from and joined
// back into st around the block (in a captured graph: two parallel branches),
// so that they share the GPU with the interior tiles instead of following
// them.  Returns the stream for list q.
struct PmlFork {
    bhfwi_ctx* c;
    hipStream_t st;
    bool on = false;
    PmlFork(bhfwi_ctx* c_, hipStream_t st_, const int na[2]) : c(c_), st(st_)
    {
        if (!c->tune.pml_overlap || na[0] <= 0 || na[1] <= 0) return;
        if (!c->pml_stream &&
            hipStreamCreateWithFlags(&c->pml_stream, hipStreamNonBlocking) != hipSuccess)
            return;
        if (!c->ev_fork && hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess)
            return;
        if (!c->ev_join && hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess)
            return;
        if (hipEventRecord(c->ev_fork, st) != hipSuccess) return;
        if (hipStreamWaitEvent(c->pml_stream, c->ev_fork, 0) != hipSuccess) return;
        on = true;
    }
    hipStream_t stream(int q) const { return (on && q == 1) ? c->pml_stream : st; }
    ~PmlFork()
    {
        if (!on) return;
        (void)hipEventRecord(c->ev_join, c->pml_stream);
        (void)hipStreamWaitEvent(st, c->ev_join, 0);
    }
};

#define BHFWI_TB(TT, RR, WW)                                                                 \
    if (T == TT && TRE == RR && W == WW) {                                                   \
        hipLaunchKernelGGL((bhfwi::k_fwd_tb<TT, RR, WW, PMV>), dim3(nact), dim3(64 * WW), 0, \
                           fork.stream(q), c->d_shots, c->ftiles.d[q], nact,                 \
                           c->tune.tile_map, n0,                                             \
                           nsteps, lam, mu, rho, wav, c->d_rec, c->d_pml_r, c->d_pml_z, in,  \
                           out, traces, hist, (long long)(2 * c->cells),                    \
                           (long long)c->cells);                                             \
        continue;                                                                            \
    }

// nsteps (<= the forward shape's T) forward steps from step n0 in LDS-tiled
// kernels: the interior tiles, then the PML sub-tiles.
void fwd_tb_launch(bhfwi_ctx* c, hipStream_t st, int n0, int nsteps, const float* lam,
                   const float* mu, const float* rho, const float* wav, const float* in,
                   float* out, float* traces, float* hist)
{
    const int na[2] = {active_tiles(c->ftiles, 0, n0), active_tiles(c->ftiles, 1, n0)};
    if (na[0] + na[1] <= 0) return;
    EvScope ev(c, st, hist ? 1 : 0);
    PmlFork fork(c, st, na);
    for (int q = 0; q < 2; ++q) {
        const int nact = na[q];
        if (nact <= 0) continue;
        const Shape sh = q ? c->ftiles.pml : fwd_shape(c);
        const int T = sh.T, TRE = sh.TRE, W = sh.W;
        if (q == 0) {
            constexpr int PMV = 0;
            BHFWI_FWD_INT(BHFWI_TB)
        } else {
            constexpr int PMV = 1;
            BHFWI_FWD_PML(BHFWI_TB)
        }
    }
}
#undef BHFWI_TB

// One adjoint block kernel with the optional outputs xm (bit 0 density, bit 1
// pseudo-Hessian) selected at run time.
template <int TT, int RR, int WW, int PMV, class... Args>
void launch_adj_tb(int xm, dim3 grid, dim3 block, hipStream_t s, Args... a)
{
    switch (xm) {
    case 1: hipLaunchKernelGGL((bhfwi::k_adj_tb<TT, RR, WW, PMV, 1>), grid, block, 0, s, a...); break;
    case 2: hipLaunchKernelGGL((bhfwi::k_adj_tb<TT, RR, WW, PMV, 2>), grid, block, 0, s, a...); break;
    case 3: hipLaunchKernelGGL((bhfwi::k_adj_tb<TT, RR, WW, PMV, 3>), grid, block, 0, s, a...); break;
    case 4: hipLaunchKernelGGL((bhfwi::k_adj_tb<TT, RR, WW, PMV, 4>), grid, block, 0, s, a...); break;
    default: hipLaunchKernelGGL((bhfwi::k_adj_tb<TT, RR, WW, PMV, 0>), grid, block, 0, s, a...); break;
    }
}

#define BHFWI_TBA(TT, RR, WW)                                                                \
    if (T == TT && TRE == RR && W == WW) {                                                   \
        launch_adj_tb<TT, RR, WW, PMV>(xm, dim3(nact), dim3(64 * WW), fork.stream(q),         \
                                       c->d_shots, ts.d[q], nact, c->tune.tile_map,          \
                                       n_hi, nsteps, lam, mu, rho, c->d_rec, resid,          \
                                       c->d_pml_r, c->d_pml_z, in, out, hist_hi,             \
                                       (long long)(2 * c->cells), acc, acc_rho, acc_h,       \
                                       c->wgrad, (long long)c->cells);                       \
        continue;                                                                            \
    }

// nsteps (<= the adjoint shape's T) adjoint steps n_hi, n_hi - 1, ... in
// LDS-tiled kernels (interior tiles, then PML sub-tiles); hist_hi is the
// history slot of step n_hi; acc_rho and acc_h (nullable) select the kernels
// that also accumulate the density correlation and the pseudo-Hessian.
void adj_tb_launch(bhfwi_ctx* c, hipStream_t st, int n_hi, int nsteps, const float* lam,
                   const float* mu, const float* rho, const float* resid, const float* in,
                   float* out, const float* hist_hi, float* acc, float* acc_rho, float* acc_h)
{
    const int xm = (acc_rho ? 1 : 0) | (acc_h ? 2 : 0) | (c->wgrad ? 4 : 0);
    const Shape xs = adj_x_shape(c);
    // the extra register sums need the alternative shape; the wavelet record does not
    const bool alt = (xm & 3) != 0 && xs.T >= 2;
    const TileSet& ts = alt ? c->xtiles : c->atiles;
    const int n_lo = n_hi - nsteps + 1;
    const int na[2] = {active_tiles(ts, 0, n_lo), active_tiles(ts, 1, n_lo)};
    if (na[0] + na[1] <= 0) return;
    EvScope ev(c, st, 2);
    PmlFork fork(c, st, na);
    for (int q = 0; q < 2; ++q) {
        const int nact = na[q];
        if (nact <= 0) continue;
        const Shape sh = q ? ts.pml : alt ? xs : adj_shape(c);
        const int T = sh.T, TRE = sh.TRE, W = sh.W;
        if (q == 0) {
            constexpr int PMV = 0;
            BHFWI_ADJ_INT(BHFWI_TBA)
        } else {
            constexpr int PMV = 1;
            BHFWI_ADJ_PML(BHFWI_TBA)
        }
    }
}
#undef BHFWI_TBA

// Adjoint steps [n0, n1) run backwards from n1 - 1 in buffers ab[*m & 1] ->
// ab[(*m + 1) & 1]; hist holds v of step n at slot n - n0.
void adj_range(bhfwi_ctx* c, hipStream_t st, int n0, int n1, const float* lam, const float* mu,
               const float* rho, const float* resid, float* const ab[2], int* m,
               const float* hist, float* acc, float* acc_rho, float* acc_h)
{
    const int64_t hslot = 2 * c->cells;
    if (c->order == 4) {
        const int T4 = c->f4.T >= 2 ? c->f4.T : 1;
        for (int n = n1 - 1; n >= n0; ++*m) {
            const int nb = std::min(T4, n - n0 + 1);
            if (T4 >= 2)
                adj4_tb_launch(c, st, n, nb, lam, mu, rho, resid, ab[*m & 1], ab[(*m + 1) & 1],
                               hist + (int64_t)(n - n0) * hslot, acc, acc_rho, acc_h);
            else
                adj4_launch(c, st, n, lam, mu, rho, resid, ab[*m & 1], ab[(*m + 1) & 1],
                            hist + (int64_t)(n - n0) * hslot, acc, acc_rho, acc_h);
            n -= nb;
        }
        return;
    }
    const Shape sh = adj_shape(c);
    if (sh.T >= 2) {
        for (int n = n1 - 1; n >= n0;) {
            const int nb = std::min(sh.T, n - n0 + 1);
            adj_tb_launch(c, st, n, nb, lam, mu, rho, resid, ab[*m & 1], ab[(*m + 1) & 1],
                          hist + (int64_t)(n - n0) * hslot, acc, acc_rho, acc_h);
            ++*m;
            n -= nb;
        }
    } else {
        for (int n = n1 - 1; n >= n0; --n, ++*m)
            adj_launch(c, st, n, lam, mu, rho, resid, ab[*m & 1], ab[(*m + 1) & 1],
                       hist + (int64_t)(n - n0) * hslot, acc, acc_rho, acc_h);
    }
}

// Forward steps [n0, n1) from buffer b[*parity] (ping-pong), one launch per
// step or tb_steps per launch; hist (nullable) receives v of step n at slot
// n - hist_base.
void fwd_range(bhfwi_ctx* c, hipStream_t st, int n0, int n1, const float* lam, const float* mu,
               const float* rho, const float* wav, float* const b[2], int* parity,
               float* traces, float* hist, int hist_base)
{
    const int64_t hslot = 2 * c->cells;
    if (c->order == 4) {
        const int T4 = c->f4.T >= 2 ? c->f4.T : 1;
        for (int n = n0; n < n1;) {
            const int nb = std::min(T4, n1 - n);
            float* h = hist ? hist + (int64_t)(n - hist_base) * hslot : nullptr;
            if (T4 >= 2)
                fwd4_tb_launch(c, st, n, nb, lam, mu, rho, wav, b[*parity], b[*parity ^ 1],
                               traces, h);
            else
                fwd4_launch(c, st, n, lam, mu, rho, wav, b[*parity], b[*parity ^ 1], traces, h);
            *parity ^= 1;
            n += nb;
        }
        return;
    }
    const int T = std::max(1, fwd_shape(c).T);
    for (int n = n0; n < n1;) {
        const int nb = std::min(T, n1 - n);
        float* h = hist ? hist + (int64_t)(n - hist_base) * hslot : nullptr;
        if (T >= 2)
            fwd_tb_launch(c, st, n, nb, lam, mu, rho, wav, b[*parity], b[*parity ^ 1], traces, h);
        else
            fwd_launch(c, st, n, lam, mu, rho, wav, b[*parity], b[*parity ^ 1], traces, h);
        *parity ^= 1;
        n += nb;
    }
}

void clear_graphs(bhfwi_ctx* c)
{
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
}

// Run `record(stream)` directly, or -- with graphs on -- capture it once per
// key on the context's private stream and replay the instantiated graph on st.
template <class F>
int run_sequence(bhfwi_ctx* c, hipStream_t st, std::vector<uintptr_t> key, F&& record)
{
    if (!c->tune.use_graph) {
        record(st);
        HIPOK(c, hipGetLastError());
        return BHFWI_OK;
    }
    key.push_back((uintptr_t)c->tune.rows_per_wave);
    key.push_back((uintptr_t)c->tune.waves_per_block);
    key.push_back((uintptr_t)c->tune.tb_steps);
    key.push_back((uintptr_t)c->tune.tb_rows);
    key.push_back((uintptr_t)c->tune.tb_waves);
    key.push_back((uintptr_t)c->tune.tile_map);
    key.push_back((uintptr_t)c->tune.adj_tb_steps);
    key.push_back((uintptr_t)c->tune.adj_tb_rows);
    key.push_back((uintptr_t)c->tune.adj_tb_waves);
    key.push_back((uintptr_t)c->tune.pml_overlap);
    key.push_back((uintptr_t)c->tune.rec_overlap);
    key.push_back((uintptr_t)c->tune.full_history);
    key.push_back((uintptr_t)c->tune.fwd_tile_overlap);
    key.push_back((uintptr_t)c->order);
    key.push_back((uintptr_t)c->f4.T);
    key.push_back((uintptr_t)c->f4.TRE);
    key.push_back((uintptr_t)c->f4.W);
    for (size_t g = 0; g < c->graphs.size(); ++g)
        if (c->graphs[g].key == key) {
            HIPOK(c, hipGraphLaunch(c->graphs[g].exec, st));
            return BHFWI_OK;
        }
    if (!c->cap_stream) HIPOK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIPOK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
    record(c->cap_stream);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
    if (e != hipSuccess || !graph)
        return fail(c, BHFWI_EHIP, "graph capture: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(c, BHFWI_EHIP, "graph instantiate: %s", hipGetErrorString(e));
    if (c->graphs.size() >= 6) {
        (void)hipGraphExecDestroy(c->graphs.front().exec);
        c->graphs.erase(c->graphs.begin());
    }
    c->graphs.push_back({std::move(key), exec});
    HIPOK(c, hipGraphLaunch(exec, st));
    return BHFWI_OK;
}

}  // namespace

extern "C" {

#ifndef BHFWI_BUILD_ID
#define BHFWI_BUILD_ID "unknown"
#endif
const char* bhfwi_build_id(void) { return BHFWI_BUILD_ID; }

int bhfwi_create(bhfwi_ctx** out, int32_t hip_device, const bhfwi_shot* shots, int32_t nshot,
                 const int32_t* rec_k, int32_t nrec_total, int64_t model_len, int32_t ckpt_every)
{
    if (!out) return BHFWI_EINVAL;
    *out = nullptr;
    bhfwi_ctx* c = new (std::nothrow) bhfwi_ctx;
    if (!c) return BHFWI_ENOMEM;
    auto bail = [&](int code) {
        g_create_err = c->err;  // readable through bhfwi_last_error(NULL)
        bhfwi_destroy(c);
        return code;
    };
    if (nshot < 1 || !shots || model_len <= 0 || ckpt_every < 1 || nrec_total < 0 ||
        (nrec_total > 0 && !rec_k))
        return bail(fail(c, BHFWI_EINVAL, "bad survey arguments"));
    c->device = hip_device;
    c->nshot = nshot;
    c->model_len = model_len;
    c->ckpt_every = ckpt_every;
    c->shots.assign(shots, shots + nshot);
    c->rec.assign(rec_k, rec_k + nrec_total);
    int64_t cell_off = 0, fst = 0, ast = 0, tr = 0, wv = 0;
    int pr_off = 0, pz_off = 0;
    std::vector<float> pmr, pmz;
    for (int s = 0; s < nshot; ++s) {
        const bhfwi_shot& h = shots[s];
        const int64_t NR = (int64_t)h.nr + h.npml_r, NZ = (int64_t)h.nz + 2 * (int64_t)h.npml_z;
        if (h.nr < 2 || h.nz < 2 || h.npml_r < 0 || h.npml_z < 0 || h.nt < 1)
            return bail(fail(c, BHFWI_EINVAL, "shot %d: bad grid sizes", s));
        if (NR * NZ >= (int64_t)1 << 31)
            return bail(fail(c, BHFWI_EINVAL, "shot %d: more than 2^31 cells", s));
        if (!(h.dr > 0) || !(h.dz > 0) || !(h.dt > 0) || !std::isfinite(h.dr) ||
            !std::isfinite(h.dz) || !std::isfinite(h.dt) || !(h.pml_vmax > 0) || !(h.f0 >= 0))
            return bail(fail(c, BHFWI_EINVAL, "shot %d: bad spacing, dt, f0 or vmax", s));
        const double cfl =
            (double)h.pml_vmax * h.dt * std::sqrt(1.0 / ((double)h.dr * h.dr) + 1.0 / ((double)h.dz * h.dz));
        if (!(cfl < 1.0))
            return bail(fail(c, BHFWI_ECFL, "shot %d: vmax dt sqrt(1/dr^2+1/dz^2) = %.4f >= 1", s, cfl));
        if (h.src_k < 0 || h.src_k >= NZ)
            return bail(fail(c, BHFWI_EINVAL, "shot %d: source row %d outside [0,%lld)", s, h.src_k,
                             (long long)NZ));
        if (h.nrec < 0 || h.rec_off < 0 || (int64_t)h.rec_off + h.nrec > nrec_total)
            return bail(fail(c, BHFWI_EINVAL, "shot %d: receiver range outside rec_k", s));
        for (int j = 0; j < h.nrec; ++j)
            if (rec_k[h.rec_off + j] < 0 || rec_k[h.rec_off + j] >= NZ)
                return bail(fail(c, BHFWI_EINVAL, "shot %d: receiver row %d outside grid", s,
                                 rec_k[h.rec_off + j]));
        {  // one receiver per row: the kernels record one trace per axial row
            std::vector<int32_t> rows(rec_k + h.rec_off, rec_k + h.rec_off + h.nrec);
            std::sort(rows.begin(), rows.end());
            for (size_t j = 1; j < rows.size(); ++j)
                if (rows[j] == rows[j - 1])
                    return bail(fail(c, BHFWI_EINVAL, "shot %d: two receivers on row %d", s,
                                     rows[j]));
        }
        if (h.model_off < 0 || h.model_ld < NZ ||
            h.model_off + (NR - 1) * h.model_ld + NZ > model_len)
            return bail(fail(c, BHFWI_EINVAL, "shot %d: model window outside the model", s));
        ShotDev S{};
        S.NR = (int)NR;
        S.NZ = (int)NZ;
        S.nr = h.nr;
        S.nz = h.nz;
        S.pr = h.npml_r;
        S.pz = h.npml_z;
        S.nt = h.nt;
        S.src_k = h.src_k;
        S.nrec = h.nrec;
        S.rec_off = h.rec_off;
        S.dr = h.dr;
        S.dz = h.dz;
        S.dt = h.dt;
        S.inv_dr = (float)(1.0 / h.dr);
        S.inv_dz = (float)(1.0 / h.dz);
        // point source spread over the on-axis cell of volume pi dr^2 dz
        S.src_scale = (float)((double)h.dt / (M_PI * (double)h.dr * h.dr * h.dz));
        S.model_off = h.model_off;
        S.model_ld = h.model_ld;
        S.psir_len = (int64_t)h.npml_r * NZ;
        S.psiz_len = NR * 2 * h.npml_z;
        const ShotLens lens = shot_lens(h);
        S.cell_off = cell_off;
        cell_off += lens.cells;
        S.fst_off = fst;
        fst += lens.fst;
        S.ast_off = ast;
        ast += lens.ast;
        S.trace_off = tr;
        tr += (int64_t)h.nrec * h.nt;
        S.wave_off = wv;
        wv += h.nt;
        S.pml_r_off = pr_off;
        S.pml_z_off = pz_off;
        pr_off += 4 * (int)NR;
        pz_off += 4 * (int)NZ;
        // PML tables: [a_int | b_int | a_half | b_half]
        const double lnR = std::log(1e-4);
        const double d0r = h.npml_r > 0 ? -3.0 * h.pml_vmax * lnR / (2.0 * h.npml_r * h.dr) : 0.0;
        const double d0z = h.npml_z > 0 ? -3.0 * h.pml_vmax * lnR / (2.0 * h.npml_z * h.dz) : 0.0;
        std::vector<float> tr_(4 * NR), tz_(4 * NZ);
        for (int i = 0; i < NR; ++i) {
            double xi = 0, xh = 0;
            if (h.npml_r > 0) {
                xi = ((double)i - h.nr) / h.npml_r;
                xh = ((double)i + 0.5 - h.nr) / h.npml_r;
            }
            pml_coef(xi, d0r, h.f0, h.dt, &tr_[i], &tr_[NR + i]);
            pml_coef(xh, d0r, h.f0, h.dt, &tr_[2 * NR + i], &tr_[3 * NR + i]);
        }
        const double lo = h.npml_z - 0.5, hi = h.npml_z + h.nz - 0.5;
        for (int k = 0; k < NZ; ++k) {
            double xi = 0, xh = 0;
            if (h.npml_z > 0) {
                const double ui = k, uh = k + 0.5;
                xi = ui < lo ? (lo - ui) / h.npml_z : (ui > hi ? (ui - hi) / h.npml_z : 0.0);
                xh = uh < lo ? (lo - uh) / h.npml_z : (uh > hi ? (uh - hi) / h.npml_z : 0.0);
            }
            pml_coef(xi, d0z, h.f0, h.dt, &tz_[k], &tz_[NZ + k]);
            pml_coef(xh, d0z, h.f0, h.dt, &tz_[2 * NZ + k], &tz_[3 * NZ + k]);
        }
        pmr.insert(pmr.end(), tr_.begin(), tr_.end());
        pmz.insert(pmz.end(), tz_.begin(), tz_.end());
        c->sd.push_back(S);
        c->nt_max = std::max(c->nt_max, h.nt);
        c->cell_steps += NR * NZ * h.nt;
    }
    c->cells = cell_off;
    c->fst_len = fst;
    c->ast_len = ast;
    c->trace_len = tr;
    c->wave_len = wv;
    c->nseg = (c->nt_max + ckpt_every - 1) / ckpt_every;
    c->tune.rows_per_wave = default_rows(c);
    c->tune.waves_per_block = 4;
    c->tune.use_graph = 1;
    c->tune.time_kernels = 0;
    c->tune.tb_steps = 6;  // measured best on single and batched shots; bhfwi_autotune refines
    c->tune.tb_rows = 32;
    c->tune.tb_waves = 16;
    c->tune.tile_map = 1;
    c->tune.pml_overlap = 0;  // measured: concurrent PML tiles crowd out interior ones
    c->tune.fwd_tile_overlap = 0;
    rebuild_work(c);

    hipError_t e = hipSetDevice(hip_device);
    if (e != hipSuccess) return bail(fail(c, BHFWI_EHIP, "hipSetDevice: %s", hipGetErrorString(e)));
#define CREATE_HIP(call)                                                                \
    do {                                                                                \
        hipError_t e2 = (call);                                                         \
        if (e2 != hipSuccess)                                                           \
            return bail(fail(c, BHFWI_EHIP, "%s: %s", #call, hipGetErrorString(e2)));   \
    } while (0)
    CREATE_HIP(hipMalloc(&c->d_shots, sizeof(ShotDev) * nshot));
    CREATE_HIP(hipMemcpy(c->d_shots, c->sd.data(), sizeof(ShotDev) * nshot, hipMemcpyHostToDevice));
    CREATE_HIP(hipMalloc(&c->d_rec, sizeof(int) * std::max(1, nrec_total)));
    if (nrec_total > 0)
        CREATE_HIP(hipMemcpy(c->d_rec, rec_k, sizeof(int) * nrec_total, hipMemcpyHostToDevice));
    CREATE_HIP(hipMalloc(&c->d_pml_r, sizeof(float) * pmr.size()));
    CREATE_HIP(hipMemcpy(c->d_pml_r, pmr.data(), sizeof(float) * pmr.size(), hipMemcpyHostToDevice));
    CREATE_HIP(hipMalloc(&c->d_pml_z, sizeof(float) * pmz.size()));
    CREATE_HIP(hipMemcpy(c->d_pml_z, pmz.data(), sizeof(float) * pmz.size(), hipMemcpyHostToDevice));
    CREATE_HIP(hipMalloc(&c->d_scratch, 4 * sizeof(float) * kPartBlocks + sizeof(double) * kPartBlocks));
    CREATE_HIP(hipMalloc(&c->d_status, sizeof(int)));
    CREATE_HIP(hipMemset(c->d_status, 0, sizeof(int)));
#undef CREATE_HIP
    if (int rc = upload_work(c)) return bail(rc);
    *out = c;
    return BHFWI_OK;
}

void bhfwi_destroy(bhfwi_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    clear_graphs(c);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->pml_stream) (void)hipStreamDestroy(c->pml_stream);
    if (c->rec_stream) (void)hipStreamDestroy(c->rec_stream);
    if (c->ev_rec_start) (void)hipEventDestroy(c->ev_rec_start);
    for (int q = 0; q < 2; ++q) {
        if (c->ev_rec[q]) (void)hipEventDestroy(c->ev_rec[q]);
        if (c->ev_adj[q]) (void)hipEventDestroy(c->ev_adj[q]);
    }
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->d_shots) (void)hipFree(c->d_shots);
    if (c->d_rec) (void)hipFree(c->d_rec);
    if (c->d_pml_r) (void)hipFree(c->d_pml_r);
    if (c->d_pml_z) (void)hipFree(c->d_pml_z);
    if (c->d_work) (void)hipFree(c->d_work);
    if (c->d_tile4) (void)hipFree(c->d_tile4);
    for (int q = 0; q < 2; ++q) {
        if (c->ftiles.d[q]) (void)hipFree(c->ftiles.d[q]);
        if (c->atiles.d[q]) (void)hipFree(c->atiles.d[q]);
        if (c->xtiles.d[q]) (void)hipFree(c->xtiles.d[q]);
        if (c->f4tiles.d[q]) (void)hipFree(c->f4tiles.d[q]);
    }
    if (c->d_scratch) (void)hipFree(c->d_scratch);
    if (c->d_status) (void)hipFree(c->d_status);
    delete c;
}

const char* bhfwi_last_error(const bhfwi_ctx* c)
{
    return c ? c->err.c_str() : g_create_err.c_str();
}

int bhfwi_sizes(const bhfwi_ctx* c, bhfwi_sizes_t* o)
{
    if (!c || !o) return BHFWI_EINVAL;
    o->fwd_ws_bytes = 2 * c->fst_len * (int64_t)sizeof(float);
    const bool full = c->tune.full_history != 0;
    o->ckpt_bytes = (full ? 2 * (int64_t)c->nt_max * c->cells
                          : (int64_t)std::max(0, c->nseg - 1) * c->fst_len) *
                    (int64_t)sizeof(float);
    const int64_t hist = full ? 0 : (c->tune.rec_overlap ? 4 : 2) * (int64_t)c->ckpt_every * c->cells;
    o->adj_ws_bytes = (2 * c->ast_len + hist) * (int64_t)sizeof(float);
    o->acc_elems = 4 * c->cells;
    o->trace_elems = c->trace_len;
    o->wavelet_elems = c->wave_len;
    o->cells = c->cells;
    o->cell_steps = c->cell_steps;
    o->nt_max = c->nt_max;
    o->ckpt_every = c->ckpt_every;
    o->nseg = c->nseg;
    o->work_items = (int32_t)c->work.size();
    return BHFWI_OK;
}

int bhfwi_plan_bytes(const bhfwi_shot* shots, int32_t nshot, int32_t ckpt_every,
                     bhfwi_plan_bytes_t* out)
{
    if (!shots || nshot < 1 || !out) {
        g_create_err = "plan_bytes: bad arguments";
        return BHFWI_EINVAL;
    }
    for (int s = 0; s < nshot; ++s)
        if (shots[s].nr < 2 || shots[s].nz < 2 || shots[s].npml_r < 0 || shots[s].npml_z < 0 ||
            shots[s].nt < 1) {
            g_create_err = "plan_bytes: bad grid sizes";
            return BHFWI_EINVAL;
        }
    std::vector<int> idx(nshot);
    for (int s = 0; s < nshot; ++s) idx[s] = s;
    const int K = ckpt_every > 0 ? ckpt_every : best_interval(shots, idx.data(), nshot);
    *out = group_bytes(shots, idx.data(), nshot, K);
    return BHFWI_OK;
}

int bhfwi_plan(const bhfwi_shot* shots, int32_t nshot, int64_t budget_bytes,
               int32_t ckpt_every, int32_t max_groups, int32_t* group_of, int32_t* ckpt_out,
               bhfwi_plan_info* info)
{
    bhfwi_plan_bytes_t probe;
    if (int rc = bhfwi_plan_bytes(shots, nshot, ckpt_every, &probe)) return rc;
    if (!group_of || !ckpt_out || !info) {
        g_create_err = "plan: null output";
        return BHFWI_EINVAL;
    }
    std::vector<int64_t> load(nshot);
    std::vector<int> order(nshot);
    int64_t trace = 0;
    for (int s = 0; s < nshot; ++s) {
        const bhfwi_shot& h = shots[s];
        load[s] = ((int64_t)h.nr + h.npml_r) * ((int64_t)h.nz + 2 * (int64_t)h.npml_z) * h.nt;
        order[s] = s;
        trace += 4 * (int64_t)h.nrec * h.nt;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return load[a] > load[b]; });
    const int64_t trace_bytes = 3 * trace;  // traces, residuals, observed data
    const int gmax = max_groups > 0 ? std::min<int>(max_groups, nshot) : nshot;
    for (int G = 1; G <= gmax; ++G) {
        std::vector<std::vector<int>> groups(G);
        std::vector<int64_t> tot(G, 0);
        for (int s : order) {
            const int g = (int)(std::min_element(tot.begin(), tot.end()) - tot.begin());
            groups[g].push_back(s);
            tot[g] += load[s];
        }
        int64_t ws[4] = {0, 0, 0, 0};
        std::vector<int> Ks;
        std::vector<std::vector<int>> used;
        for (auto& g : groups) {
            if (g.empty()) continue;
            std::sort(g.begin(), g.end());
            const int n = (int)g.size();
            const int K = ckpt_every > 0 ? ckpt_every : best_interval(shots, g.data(), n);
            const bhfwi_plan_bytes_t b = group_bytes(shots, g.data(), n, K);
            ws[0] = std::max(ws[0], b.fwd_ws_bytes);
            ws[1] = std::max(ws[1], b.ckpt_bytes);
            ws[2] = std::max(ws[2], b.adj_ws_bytes);
            ws[3] = std::max(ws[3], b.acc_bytes);
            Ks.push_back(K);
            used.push_back(g);
        }
        const int64_t wsb = ws[0] + ws[1] + ws[2] + ws[3];
        if (wsb + trace_bytes <= budget_bytes) {
            for (size_t q = 0; q < used.size(); ++q) {
                for (int s : used[q]) group_of[s] = (int32_t)q;
                ckpt_out[q] = Ks[q];
            }
            info->ngroups = (int32_t)used.size();
            info->pad_ = 0;
            info->workspace_bytes = wsb;
            info->trace_bytes = trace_bytes;
            return BHFWI_OK;
        }
    }
    g_create_err = "plan: no grouping of the shots fits the budget";
    return BHFWI_ENOMEM;
}

int bhfwi_set_tune(bhfwi_ctx* c, const bhfwi_tune* t)
{
    if (!c || !t) return BHFWI_EINVAL;
    if (t->rows_per_wave < 1 || t->use_graph < 0 || t->use_graph > 1 || t->time_kernels < 0 ||
        t->time_kernels > 1 || t->tb_steps < 0 || t->tile_map < 0 || t->tile_map > 1 ||
        t->pml_overlap < 0 || t->pml_overlap > 1 || t->rec_overlap < 0 || t->rec_overlap > 1 ||
        t->full_history < 0 || t->full_history > 1 || t->fwd_tile_overlap < 0 ||
        t->fwd_tile_overlap > 1 || (t->rec_overlap && t->pml_overlap) ||
        (t->tb_steps >= 2 && !fwd_supported(t->tb_steps, t->tb_rows, t->tb_waves)) ||
        t->adj_tb_steps < 0 ||
        (t->adj_tb_steps >= 2 && !adj_supported(t->adj_tb_steps, t->adj_tb_rows, t->adj_tb_waves)) ||
        (t->adj_tb_steps == 0 && t->tb_steps >= 2 &&
         !adj_supported(t->tb_steps, t->tb_rows, t->tb_waves)) ||
        !(t->waves_per_block == 1 || t->waves_per_block == 2 || t->waves_per_block == 4 ||
          t->waves_per_block == 8))
        return fail(c, BHFWI_EINVAL, "bad tune (rows %d, waves/block %d)", t->rows_per_wave,
                    t->waves_per_block);
    if (int rc = check_ctx(c)) return rc;
    HIPOK(c, hipDeviceSynchronize());  // no replay may still read the old work table
    clear_graphs(c);
    c->tune = *t;
    rebuild_work(c);
    return upload_work(c);
}

int bhfwi_set_order(bhfwi_ctx* c, int32_t order)
{
    if (int rc = check_ctx(c)) return rc;
    if (order != 2 && order != 4) return fail(c, BHFWI_EINVAL, "order %d: 2 or 4", order);
    // the four-point stencils lower the stability limit by 1/(|C1| + |C2|) = 6/7
    const double lim = order == 4 ? 6.0 / 7.0 : 1.0;
    for (int s = 0; s < c->nshot; ++s) {
        const bhfwi_shot& h = c->shots[s];
        const double cfl = (double)h.pml_vmax * h.dt *
                           std::sqrt(1.0 / ((double)h.dr * h.dr) + 1.0 / ((double)h.dz * h.dz));
        if (!(cfl < lim))
            return fail(c, BHFWI_ECFL, "shot %d: vmax dt sqrt(1/dr^2+1/dz^2) = %.4f >= %.4f for "
                                       "order %d", s, cfl, lim, order);
    }
    HIPOK(c, hipDeviceSynchronize());
    clear_graphs(c);
    if (order == 4 && !c->d_tile4) {
        // tiles of TI radial x TK axial cells, shot by shot
        std::vector<int> start(c->nshot + 1, 0);
        for (int s = 0; s < c->nshot; ++s) {
            const bhfwi::ShotDev& S = c->sd[s];
            start[s + 1] = start[s] + ((S.NR + bhfwi::o4::TI - 1) / bhfwi::o4::TI) *
                                          ((S.NZ + bhfwi::o4::TK - 1) / bhfwi::o4::TK);
        }
        HIPOK(c, hipMalloc(&c->d_tile4, sizeof(int) * (c->nshot + 1)));
        HIPOK(c, hipMemcpy(c->d_tile4, start.data(), sizeof(int) * (c->nshot + 1),
                           hipMemcpyHostToDevice));
        c->ntile4 = start[c->nshot];
    }
    c->order = order;
    return BHFWI_OK;
}

int bhfwi_set_order4_blocks(bhfwi_ctx* c, int32_t steps, int32_t rows, int32_t waves)
{
    if (int rc = check_ctx(c)) return rc;
    const Shape sh = steps >= 2 ? Shape{steps, rows, waves} : Shape{0, 0, 0};
    if (!f4_ok(sh))
        return fail(c, BHFWI_EINVAL, "fourth-order forward shape (%d, %d, %d) not compiled",
                    steps, rows, waves);
    HIPOK(c, hipDeviceSynchronize());
    clear_graphs(c);
    c->f4 = sh;
    rebuild_work(c);
    return upload_work(c);
}

int bhfwi_kernel_shapes(const bhfwi_ctx* c, int32_t* out)
{
    if (!c || !out) return BHFWI_EINVAL;
    const Shape xs = adj_x_shape(c);
    const bool alt = xs.T >= 2;
    const Shape s[6] = {fwd_shape(c), c->ftiles.pml, adj_shape(c), c->atiles.pml,
                        alt ? xs : adj_shape(c), alt ? c->xtiles.pml : c->atiles.pml};
    for (int q = 0; q < 6; ++q) {
        out[3 * q] = s[q].T;
        out[3 * q + 1] = s[q].TRE;
        out[3 * q + 2] = s[q].W;
    }
    return BHFWI_OK;
}

int bhfwi_autotune(bhfwi_ctx* c, void* stream, const float* lam, const float* mu,
                   const float* rho, const float* wavelet, float* traces, void* fwd_ws,
                   int64_t fwd_ws_bytes, void* adj_ws, int64_t adj_ws_bytes, float* acc,
                   int32_t probe_steps, bhfwi_tune* best, float* best_ms)
{
    if (int rc = check_ctx(c)) return rc;
    if (c->order != 2)
        return fail(c, BHFWI_EINVAL, "autotune: the fourth-order kernels have no tunable shapes");
    bhfwi_sizes_t z;
    bhfwi_sizes(c, &z);
    if (!lam || !mu || !rho || !wavelet || !traces || !fwd_ws || !adj_ws || !acc || !best)
        return fail(c, BHFWI_EINVAL, "autotune: null pointer");
    if (fwd_ws_bytes < z.fwd_ws_bytes || adj_ws_bytes < z.adj_ws_bytes)
        return fail(c, BHFWI_ENOMEM, "autotune: workspace too small");
    hipStream_t st = (hipStream_t)stream;
    const int P = std::max(1, std::min<int>(probe_steps, std::min(c->ckpt_every, c->nt_max)));
    // the probe keeps its own velocity history after the adjoint states
    if (adj_ws_bytes < (2 * c->ast_len + 2 * (int64_t)P * c->cells) * (int64_t)sizeof(float))
        return fail(c, BHFWI_ENOMEM, "autotune: adj_ws holds no history for %d probe steps "
                                     "(tune with full_history 0)", P);
    const bhfwi_tune base = c->tune;
    float* fb[2] = {(float*)fwd_ws, (float*)fwd_ws + c->fst_len};
    float* ab[2] = {(float*)adj_ws, (float*)adj_ws + c->ast_len};
    float* hist = (float*)adj_ws + 2 * c->ast_len;
    hipEvent_t e0, e1;
    HIPOK(c, hipEventCreate(&e0));
    HIPOK(c, hipEventCreate(&e1));
    auto install = [&](const bhfwi_tune& t) {
        HIPOK(c, hipStreamSynchronize(st));
        clear_graphs(c);
        c->tune = t;
        c->tune.use_graph = 0;
        c->tune.time_kernels = 0;
        rebuild_work(c);
        return upload_work(c);
    };
    auto run_fwd = [&]() {
        launch_fill(st, fb[0], 2 * c->fst_len, 0.0f);
        launch_fill(st, traces, c->trace_len, 0.0f);
        int parity = 0;
        fwd_range(c, st, 0, P, lam, mu, rho, wavelet, fb, &parity, nullptr, hist, 0);
    };
    auto run_adj = [&]() {
        launch_fill(st, ab[0], 2 * c->ast_len, 0.0f);
        int m = 0;
        adj_range(c, st, 0, P, lam, mu, rho, traces, ab, &m, hist, acc, nullptr, nullptr);
    };
    // best of repetitions 2 and 3 of `phase` (the first warms up)
    auto time_it = [&](auto&& phase, float* out, int reps) {
        float tmin = 1e30f;
        for (int rep = 0; rep < reps; ++rep) {
            HIPOK(c, hipEventRecord(e0, st));
            phase();
            HIPOK(c, hipEventRecord(e1, st));
            HIPOK(c, hipEventSynchronize(e1));
            float ms = 0.f;
            HIPOK(c, hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) tmin = std::min(tmin, ms);
        }
        *out = tmin;
        return BHFWI_OK;
    };
    // Phase 1: the forward kernel, storing the velocity history (as the
    // recompute does): one-step wave marches and every forward tile shape.
    std::vector<bhfwi_tune> cand;
    for (int r : {1, 2, 4}) {
        bhfwi_tune t = base;
        t.rows_per_wave = r;
        t.tb_steps = 0;
        t.adj_tb_steps = 0;
        cand.push_back(t);
    }
#define BHFWI_TBC(TT, RR, WW)            \
    for (int map = 0; map < 2; ++map) {  \
        bhfwi_tune t = base;             \
        t.tb_steps = TT;                 \
        t.tb_rows = RR;                  \
        t.tb_waves = WW;                 \
        t.tile_map = map;                \
        t.adj_tb_steps = 1;              \
        cand.push_back(t);               \
    }
    BHFWI_FWD_INT(BHFWI_TBC)
#undef BHFWI_TBC
    float best_f = 1e30f;
    bhfwi_tune best_tune = base;
    // every candidate with 3 repetitions, then the 4 fastest again with 6
    auto pick = [&](auto&& phase, float* best_ms_out, bhfwi_tune* best_out) {
        std::vector<std::pair<float, int>> tm;
        for (int q = 0; q < (int)cand.size(); ++q) {
            if (int rc = install(cand[q])) return rc;
            float ms;
            if (int rc = time_it(phase, &ms, 3)) return rc;
            tm.push_back({ms, q});
        }
        std::sort(tm.begin(), tm.end());
        *best_ms_out = 1e30f;
        for (int r = 0; r < (int)std::min<size_t>(4, tm.size()); ++r) {
            if (int rc = install(cand[tm[r].second])) return rc;
            float ms;
            if (int rc = time_it(phase, &ms, 6)) return rc;
            ms = std::min(ms, tm[r].first);
            if (ms < *best_ms_out) {
                *best_ms_out = ms;
                *best_out = cand[tm[r].second];
            }
        }
        return BHFWI_OK;
    };
    if (int rc = pick(run_fwd, &best_f, &best_tune)) return rc;
    // Phase 2: the adjoint with the fused correlation over the history the
    // chosen forward wrote: one step per launch and every adjoint tile shape.
    if (int rc = install(best_tune)) return rc;
    run_fwd();
    cand.clear();
    if (best_tune.tb_steps >= 2) {
        for (int r : {1, 2, 4}) {
            bhfwi_tune t = best_tune;
            t.rows_per_wave = r;
            t.adj_tb_steps = 1;
            cand.push_back(t);
        }
    } else {
        cand.push_back(best_tune);  // adjoint marches with the forward's rows
    }
#define BHFWI_TBC(TT, RR, WW)       \
    {                               \
        bhfwi_tune t = best_tune;   \
        t.adj_tb_steps = TT;        \
        t.adj_tb_rows = RR;         \
        t.adj_tb_waves = WW;        \
        cand.push_back(t);          \
    }
    BHFWI_ADJ_INT(BHFWI_TBC)
#undef BHFWI_TBC
    float best_a = 1e30f;
    bhfwi_tune best_adj = best_tune;
    if (int rc = pick(run_adj, &best_a, &best_adj)) return rc;
    best_tune = best_adj;
    const float best_t = best_f + best_a;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    clear_graphs(c);
    best_tune.use_graph = base.use_graph;
    best_tune.time_kernels = base.time_kernels;
    c->tune = best_tune;
    rebuild_work(c);
    if (int rc = upload_work(c)) return rc;
    *best = best_tune;
    if (best_ms) *best_ms = best_t;
    return BHFWI_OK;
}

int bhfwi_kernel_times(bhfwi_ctx* c, bhfwi_kernel_times_t* o, int32_t reset)
{
    if (int rc = check_ctx(c)) return rc;
    if (!o) return fail(c, BHFWI_EINVAL, "kernel_times: null output");
    HIPOK(c, hipDeviceSynchronize());
    double ms[3] = {0, 0, 0};
    int64_t cnt[3] = {0, 0, 0};
    for (auto& u : c->ev_used) {
        float t = 0.f;
        HIPOK(c, hipEventElapsedTime(&t, c->ev_pool[u.second], c->ev_pool[u.second + 1]));
        ms[u.first] += t;
        cnt[u.first] += 1;
    }
    o->fwd_ms = ms[0];
    o->rec_ms = ms[1];
    o->adj_ms = ms[2];
    o->fwd_launches = cnt[0];
    o->rec_launches = cnt[1];
    o->adj_launches = cnt[2];
    if (reset) c->ev_used.clear();
    return BHFWI_OK;
}

int bhfwi_get_tune(const bhfwi_ctx* c, bhfwi_tune* o)
{
    if (!c || !o) return BHFWI_EINVAL;
    *o = c->tune;
    return BHFWI_OK;
}

int bhfwi_moduli(void* stream, int64_t n, const float* vp, const float* vs, const float* rho,
                 float* lam, float* mu)
{
    if (n < 0 || (n > 0 && (!vp || !vs || !rho || !lam || !mu))) return BHFWI_EINVAL;
    if (n == 0) return BHFWI_OK;
    hipLaunchKernelGGL(bhfwi::k_moduli, dim3(grid1d(n)), dim3(256), 0, (hipStream_t)stream,
                       (long long)n, vp, vs, rho, lam, mu);
    return hipGetLastError() == hipSuccess ? BHFWI_OK : BHFWI_EHIP;
}

int bhfwi_moduli_grad(void* stream, int64_t n, const float* vp, const float* vs,
                      const float* rho, const float* g_lam, const float* g_mu, float* g_vp,
                      float* g_vs, float* g_rho)
{
    if (n < 0 || (n > 0 && (!vp || !vs || !rho || !g_lam || !g_mu || !g_vp || !g_vs)))
        return BHFWI_EINVAL;
    if (n == 0) return BHFWI_OK;
    hipLaunchKernelGGL(bhfwi::k_moduli_grad, dim3(grid1d(n)), dim3(256), 0, (hipStream_t)stream,
                       (long long)n, vp, vs, rho, g_lam, g_mu, g_vp, g_vs, g_rho);
    return hipGetLastError() == hipSuccess ? BHFWI_OK : BHFWI_EHIP;
}

int bhfwi_velocities(void* stream, int64_t n, const float* lam, const float* mu,
                     const float* rho, float* vp, float* vs)
{
    if (n < 0 || (n > 0 && (!vp || !vs || !rho || !lam || !mu))) return BHFWI_EINVAL;
    if (n == 0) return BHFWI_OK;
    hipLaunchKernelGGL(bhfwi::k_velocities, dim3(grid1d(n)), dim3(256), 0, (hipStream_t)stream,
                       (long long)n, lam, mu, rho, vp, vs);
    return hipGetLastError() == hipSuccess ? BHFWI_OK : BHFWI_EHIP;
}

int bhfwi_fwd_model(bhfwi_ctx* c, void* stream, const float* lam, const float* mu,
                    const float* rho, const float* wavelet, float* traces, void* fwd_ws,
                    int64_t fwd_ws_bytes, void* ckpt, int64_t ckpt_bytes, int32_t flags)
{
    if (int rc = check_ctx(c)) return rc;
    bhfwi_sizes_t z;
    bhfwi_sizes(c, &z);
    if (!lam || !mu || !rho || !wavelet || !traces || !fwd_ws)
        return fail(c, BHFWI_EINVAL, "fwd_model: null pointer");
    if (fwd_ws_bytes < z.fwd_ws_bytes)
        return fail(c, BHFWI_ENOMEM, "fwd_model: fwd_ws %lld < %lld bytes",
                    (long long)fwd_ws_bytes, (long long)z.fwd_ws_bytes);
    const bool store = (flags & BHFWI_STORE_CKPT) != 0;
    if (store && z.ckpt_bytes > 0 && (!ckpt || ckpt_bytes < z.ckpt_bytes))
        return fail(c, BHFWI_ENOMEM, "fwd_model: ckpt %lld < %lld bytes", (long long)ckpt_bytes,
                    (long long)z.ckpt_bytes);
    hipStream_t st = (hipStream_t)stream;
    float* b[2] = {(float*)fwd_ws, (float*)fwd_ws + c->fst_len};
    const int K = c->ckpt_every;
    const bool full = c->tune.full_history != 0;
    auto record = [&](hipStream_t s) {
        launch_fill(s, b[0], 2 * c->fst_len, 0.0f);
        int parity = 0;
        if (store && full) {  // the velocity history of every step, no checkpoints
            fwd_range(c, s, 0, c->nt_max, lam, mu, rho, wavelet, b, &parity, traces,
                      (float*)ckpt, 0);
            return;
        }
        for (int n = 0; n < c->nt_max; n += K) {
            const int n1 = std::min(n + K, c->nt_max);
            fwd_range(c, s, n, n1, lam, mu, rho, wavelet, b, &parity, traces, nullptr, 0);
            if (store && n1 < c->nt_max) {
                float* dst = (float*)ckpt + (int64_t)(n1 / K - 1) * c->fst_len;
                (void)hipMemcpyAsync(dst, b[parity], sizeof(float) * c->fst_len,
                                     hipMemcpyDeviceToDevice, s);
            }
        }
    };
    return run_sequence(c, st,
                        {1, (uintptr_t)lam, (uintptr_t)mu, (uintptr_t)rho, (uintptr_t)wavelet,
                         (uintptr_t)traces, (uintptr_t)fwd_ws, (uintptr_t)(store ? ckpt : nullptr)},
                        record);
}

int bhfwi_misfit(bhfwi_ctx* c, void* stream, const float* traces, const float* observed,
                 float* resid, double* J_dev, int32_t accumulate)
{
    if (int rc = check_ctx(c)) return rc;
    if (!traces || !observed || !resid || !J_dev)
        return fail(c, BHFWI_EINVAL, "misfit: null pointer");
    hipStream_t st = (hipStream_t)stream;
    const int nb = grid1d(c->trace_len, kPartBlocks);
    double* part = (double*)((float*)c->d_scratch + 4 * kPartBlocks);
    hipLaunchKernelGGL(bhfwi::k_misfit_partial, dim3(nb), dim3(256), 0, st,
                       (long long)c->trace_len, traces, observed, resid, part);
    hipLaunchKernelGGL(bhfwi::k_sum_partials, dim3(1), dim3(256), 0, st, nb, part, J_dev,
                       accumulate ? 1 : 0, c->d_status);
    HIPOK(c, hipGetLastError());
    return BHFWI_OK;
}

int bhfwi_misfit_noalloc(void* stream, int64_t n, const float* traces, const float* observed,
                         float* resid, double* J_dev, int32_t accumulate)
{
    if (n < 0 || !J_dev || (n > 0 && (!traces || !observed || !resid))) {
        g_create_err = "misfit_noalloc: negative length or null pointer";
        return BHFWI_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    int dev = -1;
    const hipError_t e = st ? hipStreamGetDevice(st, &dev) : hipGetDevice(&dev);
    if (e != hipSuccess) {
        g_create_err = std::string("misfit_noalloc: device of the stream: ") + hipGetErrorString(e);
        return BHFWI_EHIP;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        g_create_err = "misfit_noalloc: device index beyond 63";
        return BHFWI_EUNSUPPORTED;
    }
    double* part = nullptr;
    if (int rc = scratch_address(dev, &part)) return rc;
    const int nb = grid1d(n, kScratchParts);  // at most kScratchParts partial sums
    hipLaunchKernelGGL(bhfwi::k_misfit_partial, dim3(nb), dim3(256), 0, st, (long long)n, traces,
                       observed, resid, part);
    hipLaunchKernelGGL(bhfwi::k_sum_partials, dim3(1), dim3(256), 0, st, nb,
                       (const double*)part, J_dev, accumulate ? 1 : 0, (int*)nullptr);
    const hipError_t le = hipGetLastError();
    if (le != hipSuccess) {
        g_create_err = std::string("misfit_noalloc: launch: ") + hipGetErrorString(le);
        return BHFWI_EHIP;
    }
    return BHFWI_OK;
}

namespace {

// Shared body of bhfwi_adjoint_model and bhfwi_adjoint_model_density
// and bhfwi_adjoint_model_ex (acc_rho and acc_h null for the first).
int adjoint_impl(bhfwi_ctx* c, void* stream, const float* lam, const float* mu,
                 const float* rho, const float* wavelet, const float* resid, void* fwd_ws,
                 int64_t fwd_ws_bytes, const void* ckpt, int64_t ckpt_bytes, void* adj_ws,
                 int64_t adj_ws_bytes, float* acc, float* acc_rho, float* acc_h,
                 float* wgrad)
{
    if (int rc = check_ctx(c)) return rc;
    bhfwi_sizes_t z;
    bhfwi_sizes(c, &z);
    if (!lam || !mu || !rho || !wavelet || !resid || !fwd_ws || !adj_ws || !acc)
        return fail(c, BHFWI_EINVAL, "adjoint_model: null pointer");
    if (wgrad && (acc_rho || acc_h || c->order != 2))
        return fail(c, BHFWI_EUNSUPPORTED, "adjoint_model: the wavelet gradient is recorded by "
                                           "the second-order adjoint without other extra outputs");
    if (fwd_ws_bytes < z.fwd_ws_bytes || adj_ws_bytes < z.adj_ws_bytes)
        return fail(c, BHFWI_ENOMEM, "adjoint_model: workspace too small (fwd %lld/%lld, adj %lld/%lld)",
                    (long long)fwd_ws_bytes, (long long)z.fwd_ws_bytes, (long long)adj_ws_bytes,
                    (long long)z.adj_ws_bytes);
    if (z.ckpt_bytes > 0 && (!ckpt || ckpt_bytes < z.ckpt_bytes))
        return fail(c, BHFWI_ENOMEM, "adjoint_model: ckpt %lld < %lld bytes", (long long)ckpt_bytes,
                    (long long)z.ckpt_bytes);
    hipStream_t st = (hipStream_t)stream;
    float* fb[2] = {(float*)fwd_ws, (float*)fwd_ws + c->fst_len};
    float* ab[2] = {(float*)adj_ws, (float*)adj_ws + c->ast_len};
    const bool full = c->tune.full_history != 0;
    float* hist = (float*)adj_ws + 2 * c->ast_len;
    const int64_t hslot = 2 * c->cells;
    const int K = c->ckpt_every;
    float* const fbc[2] = {fb[0], fb[1]};
    const bool ovl = !full && c->tune.rec_overlap && c->nseg > 1;
    if (ovl) {
        if (!c->rec_stream)
            HIPOK(c, hipStreamCreateWithFlags(&c->rec_stream, hipStreamNonBlocking));
        if (!c->ev_rec_start)
            HIPOK(c, hipEventCreateWithFlags(&c->ev_rec_start, hipEventDisableTiming));
        for (int q = 0; q < 2; ++q) {
            if (!c->ev_rec[q]) HIPOK(c, hipEventCreateWithFlags(&c->ev_rec[q], hipEventDisableTiming));
            if (!c->ev_adj[q]) HIPOK(c, hipEventCreateWithFlags(&c->ev_adj[q], hipEventDisableTiming));
        }
    }
    // Overlapped form: the recompute of segment j (history j & 1) runs on the
    // recompute stream as soon as the adjoint of segment j + 2, the last
    // reader of that history, is done; the adjoint of segment j waits for it.
    auto record_ovl = [&](hipStream_t s) {
        hipStream_t r = c->rec_stream;
        launch_fill(s, fb[0], 2 * c->fst_len, 0.0f);
        launch_fill(s, ab[0], 2 * c->ast_len, 0.0f);
        launch_fill(s, acc, 4 * c->cells, 0.0f);
        if (acc_rho) launch_fill(s, acc_rho, 2 * c->cells, 0.0f);
        if (acc_h) launch_fill(s, acc_h, 2 * c->cells, 0.0f);
        (void)hipEventRecord(c->ev_rec_start, s);
        (void)hipStreamWaitEvent(r, c->ev_rec_start, 0);
        int m = 0;
        for (int j = c->nseg - 1; j >= 0; --j) {
            const int n0 = j * K, n1 = std::min(n0 + K, c->nt_max);
            float* h = hist + (j & 1) * 2 * (int64_t)K * c->cells;
            if (j + 2 <= c->nseg - 1) (void)hipStreamWaitEvent(r, c->ev_adj[j & 1], 0);
            if (j == 0)
                launch_fill(r, fb[0], c->fst_len, 0.0f);
            else
                (void)hipMemcpyAsync(fb[0], (const float*)ckpt + (int64_t)(j - 1) * c->fst_len,
                                     sizeof(float) * c->fst_len, hipMemcpyDeviceToDevice, r);
            int parity = 0;
            fwd_range(c, r, n0, n1, lam, mu, rho, wavelet, fbc, &parity, nullptr, h, n0);
            (void)hipEventRecord(c->ev_rec[j & 1], r);
            (void)hipStreamWaitEvent(s, c->ev_rec[j & 1], 0);
            adj_range(c, s, n0, n1, lam, mu, rho, resid, ab, &m, h, acc, acc_rho, acc_h);
            (void)hipEventRecord(c->ev_adj[j & 1], s);
        }
    };
    // Full history: the forward stored v^{n+1/2} of every step in ckpt.
    auto record_full = [&](hipStream_t s) {
        launch_fill(s, ab[0], 2 * c->ast_len, 0.0f);
        launch_fill(s, acc, 4 * c->cells, 0.0f);
        if (acc_rho) launch_fill(s, acc_rho, 2 * c->cells, 0.0f);
        if (acc_h) launch_fill(s, acc_h, 2 * c->cells, 0.0f);
        int m = 0;
        adj_range(c, s, 0, c->nt_max, lam, mu, rho, resid, ab, &m, (const float*)ckpt, acc,
                  acc_rho, acc_h);
    };
    auto record = [&](hipStream_t s) {
        if (full) {
            record_full(s);
            return;
        }
        if (ovl) {
            record_ovl(s);
            return;
        }
        launch_fill(s, fb[0], 2 * c->fst_len, 0.0f);
        launch_fill(s, ab[0], 2 * c->ast_len, 0.0f);
        launch_fill(s, acc, 4 * c->cells, 0.0f);
        if (acc_rho) launch_fill(s, acc_rho, 2 * c->cells, 0.0f);
        if (acc_h) launch_fill(s, acc_h, 2 * c->cells, 0.0f);
        int m = 0;
        for (int j = c->nseg - 1; j >= 0; --j) {
            const int n0 = j * K, n1 = std::min(n0 + K, c->nt_max);
            if (j == 0)
                launch_fill(s, fb[0], c->fst_len, 0.0f);
            else
                (void)hipMemcpyAsync(fb[0], (const float*)ckpt + (int64_t)(j - 1) * c->fst_len,
                                     sizeof(float) * c->fst_len, hipMemcpyDeviceToDevice, s);
            int parity = 0;
            fwd_range(c, s, n0, n1, lam, mu, rho, wavelet, fbc, &parity, nullptr, hist, n0);
            adj_range(c, s, n0, n1, lam, mu, rho, resid, ab, &m, hist, acc, acc_rho, acc_h);
        }
    };
    auto record_w = [&](hipStream_t s) {
        c->wgrad = wgrad;  // read by the adjoint launches while they are recorded
        if (wgrad) launch_fill(s, wgrad, c->wave_len, 0.0f);
        record(s);
        c->wgrad = nullptr;
    };
    return run_sequence(c, st,
                        {2, (uintptr_t)lam, (uintptr_t)mu, (uintptr_t)rho, (uintptr_t)wavelet,
                         (uintptr_t)resid, (uintptr_t)fwd_ws, (uintptr_t)ckpt, (uintptr_t)adj_ws,
                         (uintptr_t)acc, (uintptr_t)acc_rho, (uintptr_t)acc_h,
                         (uintptr_t)wgrad},
                        record_w);
}

}  // namespace

int bhfwi_adjoint_model(bhfwi_ctx* c, void* stream, const float* lam, const float* mu,
                        const float* rho, const float* wavelet, const float* resid,
                        void* fwd_ws, int64_t fwd_ws_bytes, const void* ckpt,
                        int64_t ckpt_bytes, void* adj_ws, int64_t adj_ws_bytes, float* acc)
{
    return adjoint_impl(c, stream, lam, mu, rho, wavelet, resid, fwd_ws, fwd_ws_bytes, ckpt,
                        ckpt_bytes, adj_ws, adj_ws_bytes, acc, nullptr, nullptr, nullptr);
}

int bhfwi_adjoint_model_density(bhfwi_ctx* c, void* stream, const float* lam, const float* mu,
                                const float* rho, const float* wavelet, const float* resid,
                                void* fwd_ws, int64_t fwd_ws_bytes, const void* ckpt,
                                int64_t ckpt_bytes, void* adj_ws, int64_t adj_ws_bytes,
                                float* acc, float* acc_rho)
{
    if (int rc = check_ctx(c)) return rc;
    if (!acc_rho) return fail(c, BHFWI_EINVAL, "adjoint_model_density: null acc_rho");
    return adjoint_impl(c, stream, lam, mu, rho, wavelet, resid, fwd_ws, fwd_ws_bytes, ckpt,
                        ckpt_bytes, adj_ws, adj_ws_bytes, acc, acc_rho, nullptr, nullptr);
}

int bhfwi_adjoint_model_ex(bhfwi_ctx* c, void* stream, const float* lam, const float* mu,
                           const float* rho, const float* wavelet, const float* resid,
                           void* fwd_ws, int64_t fwd_ws_bytes, const void* ckpt,
                           int64_t ckpt_bytes, void* adj_ws, int64_t adj_ws_bytes, float* acc,
                           float* acc_rho, float* acc_h)
{
    return adjoint_impl(c, stream, lam, mu, rho, wavelet, resid, fwd_ws, fwd_ws_bytes, ckpt,
                        ckpt_bytes, adj_ws, adj_ws_bytes, acc, acc_rho, acc_h, nullptr);
}

int bhfwi_adjoint_model_wavelet(bhfwi_ctx* c, void* stream, const float* lam, const float* mu,
                                const float* rho, const float* wavelet, const float* resid,
                                void* fwd_ws, int64_t fwd_ws_bytes, const void* ckpt,
                                int64_t ckpt_bytes, void* adj_ws, int64_t adj_ws_bytes,
                                float* acc, float* wgrad)
{
    if (int rc = check_ctx(c)) return rc;
    if (!wgrad) return fail(c, BHFWI_EINVAL, "adjoint_model_wavelet: null wgrad");
    return adjoint_impl(c, stream, lam, mu, rho, wavelet, resid, fwd_ws, fwd_ws_bytes, ckpt,
                        ckpt_bytes, adj_ws, adj_ws_bytes, acc, nullptr, nullptr, wgrad);
}

int bhfwi_gradient_hessian(bhfwi_ctx* c, void* stream, const float* acc_h, float* h_lam,
                           float* h_mu, int32_t accumulate)
{
    if (int rc = check_ctx(c)) return rc;
    if (!acc_h || !h_lam || !h_mu) return fail(c, BHFWI_EINVAL, "gradient_hessian: null pointer");
    hipStream_t st = (hipStream_t)stream;
    if (!accumulate) {
        launch_fill(st, h_lam, c->model_len, 0.0f);
        launch_fill(st, h_mu, c->model_len, 0.0f);
    }
    for (int s = 0; s < c->nshot; ++s) {
        const int64_t cells = (int64_t)c->sd[s].NR * c->sd[s].NZ;
        hipLaunchKernelGGL(bhfwi::k_window_add2, dim3(grid1d(cells)), dim3(256), 0, st,
                           c->d_shots, s, acc_h, (long long)c->cells, h_lam, h_mu);
    }
    HIPOK(c, hipGetLastError());
    return BHFWI_OK;
}

int bhfwi_gradient_density(bhfwi_ctx* c, void* stream, const float* rho, const float* acc_rho,
                           float* g_rho, int32_t accumulate)
{
    if (int rc = check_ctx(c)) return rc;
    if (!rho || !acc_rho || !g_rho) return fail(c, BHFWI_EINVAL, "gradient_density: null pointer");
    hipStream_t st = (hipStream_t)stream;
    if (!accumulate) launch_fill(st, g_rho, c->model_len, 0.0f);
    for (int s = 0; s < c->nshot; ++s) {
        const int64_t cells = (int64_t)c->sd[s].NR * c->sd[s].NZ;
        hipLaunchKernelGGL(bhfwi::k_finalize_rho_shot, dim3(grid1d(cells)), dim3(256), 0, st,
                           c->d_shots, s, rho, acc_rho, (long long)c->cells, g_rho);
    }
    HIPOK(c, hipGetLastError());
    return BHFWI_OK;
}

int bhfwi_gradient(bhfwi_ctx* c, void* stream, const float* mu, const float* acc, float* g_lam,
                   float* g_mu, float* illum, int32_t accumulate)
{
    if (int rc = check_ctx(c)) return rc;
    if (!mu || !acc || !g_lam || !g_mu || !illum)
        return fail(c, BHFWI_EINVAL, "gradient: null pointer");
    hipStream_t st = (hipStream_t)stream;
    if (!accumulate) {
        launch_fill(st, g_lam, c->model_len, 0.0f);
        launch_fill(st, g_mu, c->model_len, 0.0f);
        launch_fill(st, illum, c->model_len, 0.0f);
    }
    for (int s = 0; s < c->nshot; ++s) {
        const int64_t cells = (int64_t)c->sd[s].NR * c->sd[s].NZ;
        hipLaunchKernelGGL(bhfwi::k_finalize_shot, dim3(grid1d(cells)), dim3(256), 0, st,
                           c->d_shots, s, mu, acc, (long long)c->cells, g_lam, g_mu, illum);
    }
    HIPOK(c, hipGetLastError());
    return BHFWI_OK;
}

int bhfwi_precondition(bhfwi_ctx* c, void* stream, int64_t n, const float* illum,
                       const uint8_t* mask, float eps, float* g_lam, float* g_mu, double* gpg)
{
    if (int rc = check_ctx(c)) return rc;
    if (n < 1 || !illum || !mask || !g_lam || !g_mu || !(eps >= 0))
        return fail(c, BHFWI_EINVAL, "precondition: bad arguments");
    hipStream_t st = (hipStream_t)stream;
    const int nb = grid1d(n, kPartBlocks);
    float* part = (float*)c->d_scratch;
    hipLaunchKernelGGL(bhfwi::k_absmax_partial, dim3(nb), dim3(256), 0, st, (long long)n, mask,
                       illum, (const float*)nullptr, (const float*)nullptr,
                       (const float*)nullptr, part);
    const int na = grid1d(n, kPartBlocks);
    double* dpart = gpg ? (double*)((float*)c->d_scratch + 4 * kPartBlocks) : nullptr;
    hipLaunchKernelGGL(bhfwi::k_precond_apply, dim3(na), dim3(256), 0, st, (long long)n, mask,
                       illum, eps, part, nb, g_lam, g_mu, dpart);
    if (gpg)
        hipLaunchKernelGGL(bhfwi::k_sum_partials, dim3(1), dim3(256), 0, st, na, dpart, gpg, 0,
                           c->d_status);
    HIPOK(c, hipGetLastError());
    return BHFWI_OK;
}

int bhfwi_precondition_diag(bhfwi_ctx* c, void* stream, int64_t n, int32_t ld,
                            const float* diag, const float* row_weight, const uint8_t* mask,
                            float eps, float* g, double* gpg, int32_t accumulate)
{
    if (int rc = check_ctx(c)) return rc;
    if (n < 1 || ld < 1 || !mask || !g || !(eps >= 0))
        return fail(c, BHFWI_EINVAL, "precondition_diag: bad arguments");
    hipStream_t st = (hipStream_t)stream;
    const int nb = grid1d(n, kPartBlocks);
    float* part = (float*)c->d_scratch;
    if (diag)
        hipLaunchKernelGGL(bhfwi::k_absmax_partial, dim3(nb), dim3(256), 0, st, (long long)n,
                           mask, diag, (const float*)nullptr, (const float*)nullptr,
                           (const float*)nullptr, part);
    double* dpart = gpg ? (double*)((float*)c->d_scratch + 4 * kPartBlocks) : nullptr;
    hipLaunchKernelGGL(bhfwi::k_precond_diag_apply, dim3(nb), dim3(256), 0, st, (long long)n,
                       (int)ld, mask, diag, row_weight, eps, (const float*)part, nb, g, dpart);
    if (gpg)
        hipLaunchKernelGGL(bhfwi::k_sum_partials, dim3(1), dim3(256), 0, st, nb, dpart, gpg,
                           accumulate ? 1 : 0, c->d_status);
    HIPOK(c, hipGetLastError());
    return BHFWI_OK;
}

int bhfwi_radial_taper(void* stream, int32_t nrow, float dr, float r0, float r1, float* w)
{
    if (nrow < 1 || !w || !(dr > 0) || !(r1 >= r0)) return BHFWI_EINVAL;
    hipLaunchKernelGGL(bhfwi::k_radial_taper, dim3((nrow + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, (int)nrow, dr, r0, r1, w);
    return hipGetLastError() == hipSuccess ? BHFWI_OK : BHFWI_EHIP;
}

int bhfwi_update_density(bhfwi_ctx* c, void* stream, int64_t n, float* rho, const float* g_rho,
                         const uint8_t* mask, float eta, float rho_min, float rho_max,
                         float* alpha_out)
{
    if (int rc = check_ctx(c)) return rc;
    if (n < 1 || !rho || !g_rho || !mask || !(rho_min > 0) || !(rho_max >= rho_min))
        return fail(c, BHFWI_EINVAL, "update_density: bad arguments");
    hipStream_t st = (hipStream_t)stream;
    const int nb = grid1d(n, kPartBlocks);
    float* part = (float*)c->d_scratch;
    hipLaunchKernelGGL(bhfwi::k_absmax_partial, dim3(nb), dim3(256), 0, st, (long long)n, mask,
                       g_rho, (const float*)rho, (const float*)nullptr, (const float*)nullptr,
                       part);
    hipLaunchKernelGGL(bhfwi::k_update_density_apply, dim3(grid1d(n)), dim3(256), 0, st,
                       (long long)n, mask, rho, g_rho, (const float*)part, nb, eta, rho_min,
                       rho_max, alpha_out);
    HIPOK(c, hipGetLastError());
    return BHFWI_OK;
}

int bhfwi_status(bhfwi_ctx* c, void* stream)
{
    if (int rc = check_ctx(c)) return rc;
    HIPOK(c, hipStreamSynchronize((hipStream_t)stream));
    int h = 0;
    HIPOK(c, hipMemcpy(&h, c->d_status, sizeof(int), hipMemcpyDeviceToHost));
    if (!h) return BHFWI_OK;
    const int zero = 0;
    HIPOK(c, hipMemcpy(c->d_status, &zero, sizeof(int), hipMemcpyHostToDevice));
    return fail(c, BHFWI_ENONFINITE, "non-finite misfit or line-search slope: the traces or "
                                     "gradients hold NaN or Inf");
}

int bhfwi_line_search(bhfwi_ctx* c, void* stream, const double* J0, const double* J1,
                      const double* gpg, const float* alpha1, float* alpha_out)
{
    if (int rc = check_ctx(c)) return rc;
    if (!J0 || !J1 || !gpg || !alpha1 || !alpha_out)
        return fail(c, BHFWI_EINVAL, "line_search: null pointer");
    hipLaunchKernelGGL(bhfwi::k_line_search, dim3(1), dim3(64), 0, (hipStream_t)stream, J0, J1,
                       gpg, alpha1, alpha_out);
    HIPOK(c, hipGetLastError());
    return BHFWI_OK;
}

int bhfwi_update(bhfwi_ctx* c, void* stream, int64_t n, float* lam, float* mu, const float* rho,
                 const float* g_lam, const float* g_mu, const uint8_t* mask, float eta,
                 float alpha_override, const float* alpha_in, const bhfwi_bounds* b,
                 float* alpha_out)
{
    if (int rc = check_ctx(c)) return rc;
    if (n < 1 || !lam || !mu || !rho || !g_lam || !g_mu || !mask || !b)
        return fail(c, BHFWI_EINVAL, "update: bad arguments");
    hipStream_t st = (hipStream_t)stream;
    const int nb = grid1d(n, kPartBlocks);
    float* part = (float*)c->d_scratch;
    hipLaunchKernelGGL(bhfwi::k_absmax_partial, dim3(nb), dim3(256), 0, st, (long long)n, mask,
                       g_lam, g_mu, (const float*)lam, (const float*)mu, part);
    hipLaunchKernelGGL(bhfwi::k_update_apply, dim3(grid1d(n)), dim3(256), 0, st, (long long)n,
                       mask, lam, mu, rho, g_lam, g_mu, (const float*)part, nb, eta,
                       alpha_override, alpha_in, b->vp_min, b->vp_max, b->vs_min, b->vs_max,
                       alpha_out);
    HIPOK(c, hipGetLastError());
    return BHFWI_OK;
}

}  // extern "C"
