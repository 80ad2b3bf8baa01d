/*
 * bhfwi.h -- C-ABI of the MI355X (gfx950) hot path of gradient-descent
 * borehole acoustic full-waveform inversion
 * (Tang, Cheng, Li & Fang, "Borehole acoustic full-waveform inversion").
 *
 * The library advances the monopole velocity-stress equations in cylindrical
 * (r, z) coordinates (Method section, Eq. 2) forward and adjoint (Eq. 6),
 * correlates the two wavefields into lambda/mu gradients (Eq. 7-8), applies
 * the diagonal preconditioner and updates the model (Eq. 9-12).
 *
 * Conventions for every entry point
 *  - Return 0 on success or a negative BHFWI_E* code; bhfwi_last_error()
 *    gives the text of the last failure on that context.  Nothing throws.
 *  - Every pointer marked "device" is a HIP device pointer owned by the
 *    caller; the library never frees or retains it past the call.  Host
 *    pointers are read during the call only.
 *  - Calls are asynchronous on the given stream (hipStream_t passed as void*;
 *    NULL is the default stream).  Argument errors are reported
 *    synchronously; nothing is launched when a call fails validation.
 *  - Arrays are FP32, structure of arrays, z (k) contiguous.  A shot's padded
 *    grid has NR = nr + npml_r radial rows i and NZ = nz + 2*npml_z axial rows
 *    k; cell (i,k) of shot s reads the global model at
 *    model_off + i*model_ld + k.
 *  - Traces are packed shot after shot, each [nrec][nt]; wavelets are packed
 *    shot after shot, each [nt] sampled at t = (n + 1/2) dt.
 *
 * Staggered grid (reading of the paper's finite-difference solver): normal
 * stresses and the model at C (r=(i+1/2)dr, z=k dz), v_r at (i dr, k dz),
 * v_z at ((i+1/2)dr, (k+1/2)dz), tau_rz at (i dr, (k+1/2)dz); v_r = tau_rz = 0
 * on the axis; second order in space and time; complex-frequency-shifted PML
 * on the outer radius and both axial ends.
 */
#ifndef BHFWI_H
#define BHFWI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BHFWI_OK 0
#define BHFWI_EINVAL (-1)      /* bad shape, null pointer, geometry */
#define BHFWI_ECFL (-2)        /* time step above the stability limit */
#define BHFWI_ENOMEM (-3)      /* a workspace smaller than bhfwi_sizes() asks */
#define BHFWI_EHIP (-4)        /* HIP runtime error (text in bhfwi_last_error) */
#define BHFWI_ENONFINITE (-5)  /* non-finite values detected */
#define BHFWI_EUNSUPPORTED (-6)

typedef struct bhfwi_ctx bhfwi_ctx;

/* Identity of this build: the SHA-256 (hex) of the HIP sources and this
 * header it was compiled from.  Loaders compare it with the sources on disk
 * to refuse a stale library.  Static string; never fails. */
const char *bhfwi_build_id(void);

/* One shot (tool position), host struct. */
typedef struct {
    int32_t nr, nz;           /* physical cells, radial and axial */
    int32_t npml_r, npml_z;   /* PML cells: outer radius, each axial end */
    float dr, dz, dt;         /* m, m, s */
    int32_t nt;               /* time steps */
    float f0;                 /* Hz; PML frequency shift alpha_max = pi f0 */
    float pml_vmax;           /* m/s; PML damping d0 = -3 vmax ln(1e-4) / (2 L) */
    int32_t src_k;            /* padded-grid row of the on-axis source cell */
    int32_t nrec;             /* on-axis receivers of this shot */
    int32_t rec_off;          /* their rows are rec_k[rec_off .. rec_off+nrec) */
    int32_t pad_;             /* keep the struct 8-byte aligned; set to 0 */
    int64_t model_off;        /* global-model element of cell (0,0) */
    int64_t model_ld;         /* global-model elements between radial rows */
} bhfwi_shot;

/* Workspace sizes in bytes and packed lengths in elements for a context. */
typedef struct {
    int64_t fwd_ws_bytes;     /* forward state, double-buffered */
    int64_t ckpt_bytes;       /* forward checkpoints (one every ckpt_every steps) */
    int64_t adj_ws_bytes;     /* adjoint state, double-buffered, plus the
                                 velocity history of one checkpoint segment */
    int64_t acc_elems;        /* per-shot accumulators: 4 planes of sum(NR*NZ) */
    int64_t trace_elems;      /* sum over shots of nrec*nt */
    int64_t wavelet_elems;    /* sum over shots of nt */
    int64_t cells;            /* sum over shots of NR*NZ */
    int64_t cell_steps;       /* sum over shots of NR*NZ*nt */
    int32_t nt_max;
    int32_t ckpt_every;
    int32_t nseg;             /* checkpoint segments of the longest shot */
    int32_t work_items;       /* wave work items per time step */
} bhfwi_sizes_t;

/* Tunables of the wave-march kernels (every value in range is correct; only
 * speed changes).  rows_per_wave <= 4 selects kernels that issue all loads of
 * a wave before computing. */
typedef struct {
    int32_t rows_per_wave;    /* radial rows one wave marches per launch, >= 1 */
    int32_t waves_per_block;  /* 1, 2, 4 or 8 wave64 per workgroup */
    int32_t use_graph;        /* 1: capture each call's launch sequence once per
                                 set of pointers as a HIP graph and replay it;
                                 0: launch step by step from the host */
    int32_t time_kernels;     /* 1 (with use_graph 0): bracket every time-step
                                 kernel with a pair of HIP events on its stream;
                                 read the sums with bhfwi_kernel_times */
    int32_t tb_steps;         /* >= 2: forward and recompute steps run
                                 T = tb_steps at a time in LDS-tiled kernels;
                                 0 or 1: one step per launch (wave march) */
    int32_t tb_rows;          /* radial rows of a tile including its halo */
    int32_t tb_waves;         /* wave64 per tile workgroup (4, 8 or 16).  Supported
                                 (tb_steps, tb_rows, tb_waves): (2|3|4, 16, 4),
                                 (2|3|4, 16, 8), (2|3|4|6, 24, 8),
                                 (4|6|8, 32, 8), (2|3|4, 16, 16),
                                 (4|6|8, 32, 16), (4|6|8, 48, 16), (4|8, 64, 16).
                                 Tiles that touch a PML layer run a kernel
                                 that carries the PML memories; for the 64-row
                                 shapes they are cut into sub-tiles of a
                                 smaller shape with the same T
                                 (bhfwi_kernel_shapes reports it) */
    int32_t tile_map;         /* order of the tiles of a temporally blocked launch:
                                 0: axial tile fastest, workgroups in table order;
                                 1: radial tile fastest, and each of the 8 XCDs of
                                 the GPU walks one contiguous chunk of the table
                                 so that tiles with overlapping halos share its L2 */
    int32_t adj_tb_steps;     /* adjoint: 0 = the forward's shape (tb_*), 1 = one
                                 step per launch (wave march), >= 2 = its own
                                 shape (adj_tb_steps, adj_tb_rows, adj_tb_waves)
                                 from the supported forward shapes except
                                 (4, 64, 16); PML tiles of the 48- and 64-row
                                 shapes run as sub-tiles of a smaller shape,
                                 and with extra outputs 8x64x16 runs as
                                 8x48x16 (bhfwi_kernel_shapes) */
    int32_t adj_tb_rows;
    int32_t adj_tb_waves;
    int32_t pml_overlap;      /* 1: the PML tiles of a time block run on a second
                                 stream alongside the interior tiles (forked and
                                 joined around the block); 0 (default): after
                                 them on the caller's stream */
    int32_t rec_overlap;      /* 1: bhfwi_adjoint_model recomputes checkpoint
                                 segment j-1 on a second stream while the adjoint
                                 of segment j runs (two velocity histories:
                                 adj_ws_bytes grows by 8 ckpt_every cells bytes;
                                 query bhfwi_sizes after setting it); the results
                                 are bit-identical to 0 (default).  Not combined
                                 with pml_overlap. */
    int32_t full_history;     /* 1: no checkpoints and no recompute: the forward
                                 of bhfwi_fwd_model with BHFWI_STORE_CKPT writes
                                 v^{n+1/2} of every step into ckpt (ckpt_bytes
                                 becomes 8 nt_max cells bytes; adj_ws_bytes
                                 drops its history) and bhfwi_adjoint_model reads
                                 it there.  For surveys whose whole history fits
                                 in HBM; rec_overlap then has nothing to do.
                                 Gradients equal the checkpointed ones to FP32
                                 regrouping of the correlation sums. */
    int32_t fwd_tile_overlap; /* 1: the forward's temporally blocked launches add,
                                 in every column clear of the axial PML, one
                                 interior tile that ends where the radial PML
                                 layer's halo begins; its window overlaps the
                                 interior tile below it and it writes back only
                                 the rows above that tile, so that the PML tiles
                                 cover fewer rows; pays on launches of many rounds of
                                 workgroups.  0 (default): interior tiles stop
                                 at the first one whose halo reaches the layer.
                                 Traces and gradients differ from 0 only by FP32
                                 rounding (rows move between the interior and
                                 the PML kernel). */
} bhfwi_tune;

/* Memory of one group of shots evaluated together (bhfwi_plan_bytes). */
typedef struct {
    int32_t ckpt_every;       /* checkpoint interval the figures are for */
    int32_t pad_;
    int64_t fwd_ws_bytes, ckpt_bytes, adj_ws_bytes, acc_bytes;  /* as bhfwi_sizes */
    int64_t total_bytes;      /* their sum */
} bhfwi_plan_bytes_t;

/* Result of bhfwi_plan. */
typedef struct {
    int32_t ngroups;
    int32_t pad_;
    int64_t workspace_bytes;  /* workspaces shared by the groups: per kind the
                                 maximum over groups, summed over kinds */
    int64_t trace_bytes;      /* traces, residuals and observed data of all shots */
} bhfwi_plan_info;

/* Per-kernel time sums collected while tune.time_kernels is on: the forward
 * step of bhfwi_fwd_model, the recompute step (forward step storing v) and
 * the adjoint step of bhfwi_adjoint_model.  Synchronises the device. */
typedef struct {
    double fwd_ms, rec_ms, adj_ms;
    int64_t fwd_launches, rec_launches, adj_launches;
} bhfwi_kernel_times_t;

/* Create a context for a survey: a set of shots over one global model of
 * model_len elements.  rec_k (host, nrec_total entries) holds the receiver
 * rows of every shot.
 * ckpt_every > 0 is the forward checkpoint interval in steps.  Validates the
 * geometry (receiver and source rows inside the grid, at most one receiver
 * per row of a shot, windows inside the model) and the CFL condition vmax dt sqrt(1/dr^2 + 1/dz^2) < 1 with vmax =
 * pml_vmax.  Uploads the shot table, receiver rows and PML profiles to the
 * device selected by hip_device. */
int bhfwi_create(bhfwi_ctx **out, int32_t hip_device, const bhfwi_shot *shots, int32_t nshot,
                 const int32_t *rec_k, int32_t nrec_total, int64_t model_len,
                 int32_t ckpt_every);
void bhfwi_destroy(bhfwi_ctx *ctx);
/* Text of the last failure on ctx; with ctx == NULL, of the last failed
 * bhfwi_create on this thread. */
const char *bhfwi_last_error(const bhfwi_ctx *ctx);
int bhfwi_sizes(const bhfwi_ctx *ctx, bhfwi_sizes_t *out);
/* Spatial order of the step, 2 (default) or 4.  The paper names its
 * finite-difference scheme only by citation; order 4 replaces every staggered
 * difference and two-point 1/r average by its four-point form,
 * D f = [9/8 (f(+1/2) - f(-1/2)) - 1/24 (f(+3/2) - f(-3/2))] / h and
 * I f = 9/16 (f(+1/2) + f(-1/2)) - 1/16 (f(+3/2) + f(-3/2)), with the fields
 * mirrored across the axis (even at half radial positions, odd at integer
 * ones), and the on-axis source divided by the axis cell's weight sqrt(6/7)
 * in the norm in which that divergence conserves flux.  Applies to
 * bhfwi_fwd_model and the bhfwi_adjoint_model family, the density and
 * pseudo-Hessian outputs included (no autotune; time blocks set by
 * bhfwi_set_order4_blocks).  Order 4 needs the stricter stability bound
 * vmax dt sqrt(1/dr^2 + 1/dz^2) < 6/7 (BHFWI_ECFL otherwise).  Synchronises
 * the device. */
int bhfwi_set_order(bhfwi_ctx *ctx, int32_t order);
/* Time blocks of the fourth-order step (bhfwi_set_order(4)): the forward and
 * the adjoint (with the Eq. 7-8 correlation, the density correlation and the
 * pseudo-Hessian where they are asked for) advance `steps` steps per launch on workgroups of `waves` wave64 whose window is 64 axial by
 * `rows` radial cells with a 3*steps-cell halo (each step reaches three cells
 * on either side).  steps < 2 runs one step per launch.  The compiled shape is
 * (2, 32, 16), the default; others give BHFWI_EINVAL.  Results equal the
 * one-step kernels' to FP32 rounding.  Synchronises the device. */
int bhfwi_set_order4_blocks(bhfwi_ctx *ctx, int32_t steps, int32_t rows, int32_t waves);
int bhfwi_set_tune(bhfwi_ctx *ctx, const bhfwi_tune *tune);
int bhfwi_get_tune(const bhfwi_ctx *ctx, bhfwi_tune *out);
/* Autotuner: times, on this survey, every forward kernel shape (one-step wave
 * marches of 1, 2 and 4 rows per wave, every temporally blocked shape in both
 * tile maps) over probe_steps forward steps storing the velocity history from
 * a zero state and keeps the fastest; then every adjoint shape (marches and
 * tiles) over the same steps driven by a zero residual.  Installs the result
 * as the context's tune, copies it to *best (host) and the sum of the two
 * probe times to *best_ms (host).  probe_steps is clamped to
 * [1, min(ckpt_every, nt)].
 * traces (trace_elems floats), fwd_ws, adj_ws and acc are scratch; their
 * contents are overwritten.  Synchronises the stream. */
int bhfwi_autotune(bhfwi_ctx *ctx, void *stream, const float *lam, const float *mu,
                   const float *rho, const float *wavelet, float *traces, void *fwd_ws,
                   int64_t fwd_ws_bytes, void *adj_ws, int64_t adj_ws_bytes, float *acc,
                   int32_t probe_steps, bhfwi_tune *best, float *best_ms);

/* HBM planner (host only; no device is touched).  One-level checkpointing
 * of a group keeps ceil(nt_max/K) - 1 forward states of F floats and the
 * velocity history of one K-step segment (2 K C floats for C cells), least
 * near K = sqrt(nt_max F / (2 C)).
 * bhfwi_plan_bytes: the workspace bytes of shots[0..nshot) as one context with
 * interval ckpt_every, or with the memory-optimal multiple of 8 when
 * ckpt_every <= 0 (the figures bhfwi_sizes reports for such a context).
 * bhfwi_plan: splits the shots into the fewest groups (at most max_groups;
 * <= 0: nshot), balanced longest-processing-time first on NR NZ nt, whose
 * shared workspaces plus all trace buffers fit budget_bytes.  Outputs (host):
 * group_of[s] for every shot (groups numbered from 0), ckpt_out[g] for every
 * group (nshot entries suffice), *info.  BHFWI_ENOMEM when even nshot groups
 * do not fit; BHFWI_EINVAL on bad sizes.  Text via bhfwi_last_error(NULL). */
int bhfwi_plan_bytes(const bhfwi_shot *shots, int32_t nshot, int32_t ckpt_every,
                     bhfwi_plan_bytes_t *out);
int bhfwi_plan(const bhfwi_shot *shots, int32_t nshot, int64_t budget_bytes,
               int32_t ckpt_every, int32_t max_groups, int32_t *group_of, int32_t *ckpt_out,
               bhfwi_plan_info *info);

/* The temporally blocked kernel shapes the current tune runs, 18 int32 to
 * out (host): (T, rows, waves) of the forward kernel on tiles clear of the
 * PML, of the forward kernel on the PML sub-tiles, the same two for the
 * adjoint, and the same two for the adjoint with extra outputs
 * (bhfwi_adjoint_model_ex): an interior adjoint shape with four rows per
 * thread runs those as the shape with three rows per thread, same T and
 * waves (8x64x16 -> 8x48x16), whose registers hold the extra sums; T = 0
 * where that part runs one step per launch. */
int bhfwi_kernel_shapes(const bhfwi_ctx *ctx, int32_t *out);

/* Read (and with reset != 0 clear) the sums of bhfwi_kernel_times_t. */
int bhfwi_kernel_times(bhfwi_ctx *ctx, bhfwi_kernel_times_t *out, int32_t reset);

/* ---- Starting model (Introduction; Numerical Examples section, Fig. 3-4):
 * the paper starts its inversions from velocities picked by semblance
 * analysis of the array waveforms -- near-source data for the formation at
 * the wall, far-source data for the formation 1 m away -- interpolated
 * linearly in radius.  These calls do not need a context. */

/* Slowness-time coherence of ngather receiver gathers (device arrays):
 * traces [g][nrec][nt] (nrec <= 64), offset [g][nrec] (m, axial distance of
 * each receiver from the gather's first), slownesses p0 + j dp (s/m),
 * j < np, windows of win (<= 2048) samples starting at sample i*tau_stride,
 * i < ntau.  coh [g][np][ntau] (device, overwritten) =
 *   sum_window (sum_m x_m(n + p off_m/dt))^2 / (nrec sum_window sum_m x_m^2),
 * with each receiver read p*off_m/dt samples later, linearly interpolated
 * between samples and zero outside its record; 0 for a window without
 * energy.  energy (nullable, same shape) receives the window energy
 * sum_window sum_m x_m^2.
 * FP32 data, interpolation, stack and energy; window sums in double (as
 * differences of prefix sums).  Returns BHFWI_EINVAL on bad sizes. */
int bhfwi_semblance(void *stream, int32_t ngather, int32_t nrec, int32_t nt,
                    const float *traces, float dt, const float *offset, int32_t np, float p0,
                    float dp, int32_t ntau, int32_t tau_stride, int32_t win, float *coh,
                    float *energy);
/* Per gather, the slowness of the largest coherence among slownesses in
 * [lo, p_hi], lo = max(p_lo, ref_scale * p_ref[g]) when p_ref (device,
 * ngather) is given (e.g. the S band above a multiple of the picked P
 * slowness), over the windows whose energy (the map bhfwi_semblance writes;
 * nullable: all windows) is at least rel_floor times the gather's largest;
 * ties go to the smaller slowness.  proj (device, [ngather][np], written):
 * per slowness the largest coherence over those windows (-1 if none), the
 * coherence-versus-slowness projection.  p_out, c_out: device, ngather
 * floats (0 and 0 if the band holds no slowness). */
int bhfwi_semblance_pick(void *stream, int32_t ngather, int32_t np, int32_t ntau,
                         const float *coh, const float *energy, float rel_floor, float p0,
                         float dp, const float *p_ref, float ref_scale, float p_lo, float p_hi,
                         float *proj, float *p_out, float *c_out);
/* Starting velocities on an NR x NZ grid (device): per axial row k, the wall
 * values vp_wall[k], vs_wall[k] at r = a, the far values vp_far[k],
 * vs_far[k] at r = a + dist, linear in r = (i + 1/2) dr between and constant
 * beyond; cells with r < a take vp_fluid and vs = 0. */
int bhfwi_starting_model(void *stream, int32_t NR, int32_t NZ, float dr, float a, float dist,
                         const float *vp_wall, const float *vs_wall, const float *vp_far,
                         const float *vs_far, float vp_fluid, float *vp, float *vs);

/* Eq. 3-4 (Method section): lam = rho vp^2 - 2 rho vs^2, mu = rho vs^2,
 * n elements, device arrays. */
int bhfwi_moduli(void *stream, int64_t n, const float *vp, const float *vs, const float *rho,
                 float *lam, float *mu);
/* Chain rule of Eq. 3-4 for a velocity parameterisation:
 * g_vp = 2 rho vp g_lam, g_vs = 2 rho vs (g_mu - 2 g_lam); n elements, device.
 * g_rho (nullable; overwritten) receives the moduli's share of dJ/drho at
 * fixed velocities, (vp^2 - 2 vs^2) g_lam + vs^2 g_mu, to be added to the
 * buoyancy part from bhfwi_gradient_density for a (vp, vs, rho) inversion. */
int bhfwi_moduli_grad(void *stream, int64_t n, const float *vp, const float *vs,
                      const float *rho, const float *g_lam, const float *g_mu, float *g_vp,
                      float *g_vs, float *g_rho);
/* Eq. 11-12: vp = sqrt((lam + 2 mu)/rho), vs = sqrt(mu/rho). */
int bhfwi_velocities(void *stream, int64_t n, const float *lam, const float *mu,
                     const float *rho, float *vp, float *vs);

#define BHFWI_STORE_CKPT 1

/* Forward modelling (Eq. 2) of every shot.  Device inputs: lam, mu, rho
 * (global model), wavelet (packed).  Device output: traces (packed), the mean
 * normal stress at each receiver after each step (Method section: pressure
 * recorded in the fluid).  fwd_ws (>= fwd_ws_bytes) is scratch for the state.
 * With BHFWI_STORE_CKPT, ckpt (>= ckpt_bytes) receives the state every
 * ckpt_every steps for bhfwi_adjoint_model, or, with the tune's
 * full_history, the velocities v^{n+1/2} of every step. */
int bhfwi_fwd_model(bhfwi_ctx *ctx, void *stream, const float *lam, const float *mu,
                    const float *rho, const float *wavelet, float *traces, void *fwd_ws,
                    int64_t fwd_ws_bytes, void *ckpt, int64_t ckpt_bytes, int32_t flags);

/* Eq. 1 and 5: resid = traces - observed (packed), and J = 0.5 sum resid^2
 * summed in double (deterministic two-level reduction) into *J_dev (device):
 * overwritten, or added to when accumulate != 0 (several shot groups). */
int bhfwi_misfit(bhfwi_ctx *ctx, void *stream, const float *traces, const float *observed,
                 float *resid, double *J_dev, int32_t accumulate);

/* bhfwi_misfit for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * no context, and no hipMalloc, hipFree or allocating library call.  Same
 * arithmetic and outputs as bhfwi_misfit on n packed samples: resid (device,
 * n) = traces - observed, and 0.5 sum resid^2 summed in double into *J_dev
 * (device; overwritten, or added to when accumulate != 0).  The partial sums
 * live in a fixed device array of the library (1024 doubles, one copy per
 * GPU, held until the process ends); n may be any length >= 0, since the
 * first pass never uses more than 1024 blocks.  The device is the stream's
 * (NULL: the current device), index at most 63.  Calls that overlap on one
 * GPU share that array and race: serialise them (one stream, or events).
 * Returns EINVAL for n < 0 or a null pointer, EUNSUPPORTED for a device
 * index above 63, EHIP for a runtime error; text in bhfwi_last_error(NULL).
 * No device status word: a non-finite sum shows as a non-finite *J_dev. */
int bhfwi_misfit_noalloc(void *stream, int64_t n, const float *traces, const float *observed,
                         float *resid, double *J_dev, int32_t accumulate);

/* Adjoint modelling (Eq. 6, as the exact transpose of the discrete forward)
 * driven by resid = dJ/dtraces (packed), fused with the zero-lag correlation
 * of Eq. 7-8.  Each checkpoint segment is recomputed from ckpt (written by
 * bhfwi_fwd_model with BHFWI_STORE_CKPT and the same model) storing v, then
 * run backwards (with the tune's full_history, ckpt already holds v of every
 * step and nothing is recomputed).  acc (device, acc_elems floats, overwritten) receives per
 * shot, on the shot's padded grid: plane 0 dJ/dlambda, plane 1 the C-node
 * part of dJ/dmu, plane 2 dJ/dmu_S at tau_rz nodes, plane 3 the illumination
 * sum_n dt |v|^2.  adj_ws (>= adj_ws_bytes) is scratch. */
int bhfwi_adjoint_model(bhfwi_ctx *ctx, void *stream, const float *lam, const float *mu,
                        const float *rho, const float *wavelet, const float *resid,
                        void *fwd_ws, int64_t fwd_ws_bytes, const void *ckpt,
                        int64_t ckpt_bytes, void *adj_ws, int64_t adj_ws_bytes, float *acc);

/* bhfwi_adjoint_model plus the gradient with respect to the source wavelet
 * (an extension: the paper's source is a known Ricker).  The source adds
 * src_scale w[n] to the three normal stresses of the on-axis source cell in
 * step n (src_scale = dt / (pi dr^2 dz)), so dJ/dw[n] = src_scale times the
 * sum of the three adjoint normal stresses there, dJ/dtau^{n+1}: the
 * transpose of the linear map wavelet -> traces applied to resid.  acc as
 * for bhfwi_adjoint_model; wgrad (device, wavelet_elems floats, packed like
 * the wavelets, overwritten, not null).  Second order only: EUNSUPPORTED
 * after bhfwi_set_order(4).  Same cost as bhfwi_adjoint_model. */
int bhfwi_adjoint_model_wavelet(bhfwi_ctx *ctx, void *stream, const float *lam,
                                const float *mu, const float *rho, const float *wavelet,
                                const float *resid, void *fwd_ws, int64_t fwd_ws_bytes,
                                const void *ckpt, int64_t ckpt_bytes, void *adj_ws,
                                int64_t adj_ws_bytes, float *acc, float *wgrad);

/* Gradient finalize of Eq. 7-8 (the lambda and mu gradients, with the misfit
 * of Eq. 1 summed over shots).  Eq. 8's tau_rz term is correlated at the
 * tau_rz nodes, whose rigidity is the harmonic mean of the four surrounding
 * cells (zero if any of them is fluid); this call folds that node gradient
 * into the C cells by the chain rule d mu_S / d mu_c = mu_S^2 / (4 mu_c^2)
 * for each occurrence of c (cells with mu = 0 keep only their own term), and
 * sums every shot's window into the global model grid in shot order (no
 * atomics; deterministic).  mu (device, model_len) is the model the adjoint
 * ran on; acc (device, acc_elems) is bhfwi_adjoint_model's output.  Outputs
 * (device, model_len each): g_lam, g_mu, illum -- overwritten, or added to
 * when accumulate != 0 (contexts holding further groups of shots of one
 * model).  Cells outside every shot's window receive 0 (or keep their value
 * when accumulating).  EINVAL on a null pointer. */
int bhfwi_gradient(bhfwi_ctx *ctx, void *stream, const float *mu, const float *acc,
                   float *g_lam, float *g_mu, float *illum, int32_t accumulate);

/* bhfwi_adjoint_model plus the density gradient.  The paper inverts lambda
 * and mu with the density held fixed (Method section); this extension
 * differentiates the misfit through the buoyancies of the velocity update of
 * Eq. 2 as well, for joint inversion.  acc as for bhfwi_adjoint_model;
 * acc_rho (device, 2 * cells floats, overwritten, not null) receives per shot
 * b dJ/db at the v_r nodes (plane 0) and at the v_z nodes (plane 1), b the
 * buoyancy of that node.  Same cost as bhfwi_adjoint_model plus two
 * multiply-adds per node and step; no further history is stored. */
int bhfwi_adjoint_model_density(bhfwi_ctx *ctx, void *stream, const float *lam,
                                const float *mu, const float *rho, const float *wavelet,
                                const float *resid, void *fwd_ws, int64_t fwd_ws_bytes,
                                const void *ckpt, int64_t ckpt_bytes, void *adj_ws,
                                int64_t adj_ws_bytes, float *acc, float *acc_rho);

/* bhfwi_adjoint_model with optional extra outputs, each selected by a
 * non-null pointer (device, 2 * cells floats, overwritten, per shot on the
 * shot's padded grid):
 *   acc_rho  the density correlation, as for bhfwi_adjoint_model_density;
 *   acc_h    the virtual-source pseudo-Hessian diagonal, an alternative to the
 *            illumination as the diagonal of the preconditioner (the paper
 *            gives that preconditioner only as diagonal, Numerical Examples
 *            section, Fig. 6): the squared derivative of the stress update with
 *            respect to each modulus applied to the forward wavefield, summed
 *            over steps.  With the strain rates of v^{n+1/2} at C cell (i,k),
 *            plane 0 H_lambda = sum_n 3 dt^2 (e_rr + e_tt + e_zz)^2 and plane 1
 *            H_mu = sum_n dt^2 (4 (e_rr^2 + e_tt^2 + e_zz^2) + (e_z + e_r)^2),
 *            the last from the tau_rz node (i,k) (i >= 1).
 * Each extra output adds two multiply-adds per node and step to the adjoint
 * kernels; no further history is stored.  Where the tune names an adjoint
 * shape with four rows per thread, these launches run on the tiles of the
 * shape with three (bhfwi_kernel_shapes, entries 4 and 5). */
int bhfwi_adjoint_model_ex(bhfwi_ctx *ctx, void *stream, const float *lam, const float *mu,
                           const float *rho, const float *wavelet, const float *resid,
                           void *fwd_ws, int64_t fwd_ws_bytes, const void *ckpt,
                           int64_t ckpt_bytes, void *adj_ws, int64_t adj_ws_bytes, float *acc,
                           float *acc_rho, float *acc_h);

/* Sums every shot's window of acc_h (from bhfwi_adjoint_model_ex) into the
 * global grids h_lam and h_mu (device, model_len) in shot order:
 * overwritten, or added to when accumulate != 0. */
int bhfwi_gradient_hessian(bhfwi_ctx *ctx, void *stream, const float *acc_h, float *h_lam,
                           float *h_mu, int32_t accumulate);

/* Density gradient finalize: with b_R = 2/(rho[i-1,k] + rho[i,k]) and
 * b_Z = 2/(rho[i,k] + rho[i,k1]), k1 = min(k+1, NZ-1), every node adds
 * -(b/2) (b dJ/db) to each of its two cells; gathered per cell and summed
 * over shots in shot order (deterministic).  g_rho (device, model_len)
 * overwritten, or added to when accumulate != 0. */
int bhfwi_gradient_density(bhfwi_ctx *ctx, void *stream, const float *rho,
                           const float *acc_rho, float *g_rho, int32_t accumulate);

/* Diagonal preconditioner (Numerical Examples section, Fig. 6): with
 * E = illum and Emax its maximum over mask cells, g <- g / (E + eps Emax) for
 * lam and mu on mask cells, 0 elsewhere.  n elements, device arrays;
 * mask is uint8 (1 = invert this cell).  gpg (device double, nullable)
 * receives sum over mask cells of g . P g for both parameters, taken before
 * the scaling (deterministic two-level sum): minus the slope of the misfit
 * along the preconditioned step, as bhfwi_line_search needs it. */
int bhfwi_precondition(bhfwi_ctx *ctx, void *stream, int64_t n, const float *illum,
                       const uint8_t *mask, float eps, float *g_lam, float *g_mu, double *gpg);

/* One gradient through a general diagonal preconditioner (alternatives to
 * the illumination of bhfwi_precondition; the paper fixes only that it is
 * diagonal and suppresses the near-wall guided waves, Fig. 6):
 * g <- w[c / ld] g / (d + eps max d) on mask cells, 0 elsewhere, with d =
 * diag (nullable: the factor is then 1; max over mask cells) and w =
 * row_weight (nullable: 1), one weight per radial row of ld elements (a
 * radial taper).  n elements, device arrays.  gpg (device double, nullable)
 * receives sum over mask cells of g . P g taken before the scaling,
 * overwritten, or added to when accumulate != 0 (one call per parameter). */
int bhfwi_precondition_diag(bhfwi_ctx *ctx, void *stream, int64_t n, int32_t ld,
                            const float *diag, const float *row_weight, const uint8_t *mask,
                            float eps, float *g, double *gpg, int32_t accumulate);

/* Radial taper for bhfwi_precondition_diag: w[i] for the nrow radial rows of
 * C cells, r = (i + 1/2) dr: 0 for r <= r0, sin^2(pi/2 (r - r0)/(r1 - r0))
 * between, 1 for r >= r1 (a step at r0 when r1 == r0).  It mutes the gradient
 * next to the borehole wall, where the guided waves dominate it.  w device,
 * nrow floats. */
int bhfwi_radial_taper(void *stream, int32_t nrow, float dr, float r0, float r1, float *w);

/* Density step of a joint inversion (the paper keeps the density fixed):
 * the greatest-change rule applied to the density on its own,
 * alpha = eta max|rho| / max|g_rho| over mask cells, then
 * rho <- clamp(rho - alpha g_rho, rho_min, rho_max) on mask cells.  n
 * elements, device arrays; alpha_out (device float, nullable) receives alpha.
 * Call before bhfwi_update so that its velocity bounds use the new density. */
int bhfwi_update_density(bhfwi_ctx *ctx, void *stream, int64_t n, float *rho,
                         const float *g_rho, const uint8_t *mask, float eta, float rho_min,
                         float rho_max, float *alpha_out);

/* Device-side status: synchronises the stream and returns BHFWI_ENONFINITE
 * (text via bhfwi_last_error) if any bhfwi_misfit or bhfwi_precondition
 * since the last call met a non-finite sum (NaN or Inf in the traces or the
 * gradients), clearing the flag; BHFWI_OK otherwise. */
int bhfwi_status(bhfwi_ctx *ctx, void *stream);

/* Step length of a parabolic line search along the preconditioned gradient
 * (Eq. 9-10; the paper leaves the step rule open beyond letting alpha bound
 * the greatest change).  Inputs, all device scalars: J0 the misfit of the
 * current model, J1 the misfit after a trial update of length alpha1 (the
 * greatest-change rule of bhfwi_update), gpg from bhfwi_precondition.  The
 * parabola through J0 with slope -gpg and through J1 gives
 * alpha = gpg alpha1^2 / (2 (J1 - J0 + gpg alpha1)), clamped to
 * [alpha1/10, 3 alpha1] when that curvature is positive; otherwise alpha =
 * alpha1 if J1 <= J0, else alpha1/2.  alpha1 <= 0 gives 0.  Writes alpha_out
 * (device float) without synchronising. */
int bhfwi_line_search(bhfwi_ctx *ctx, void *stream, const double *J0, const double *J1,
                      const double *gpg, const float *alpha1, float *alpha_out);

/* Velocity box applied after the update. */
typedef struct {
    float vp_min, vp_max, vs_min, vs_max;
} bhfwi_bounds;

/* Eq. 9-10 on mask cells: lam -= alpha g_lam, mu -= alpha g_mu, with one
 * alpha = eta / max(max|g_lam|/max|lam|, max|g_mu|/max|mu|) over mask cells
 * (the step controls the greatest change), or alpha = alpha_override when it
 * is > 0, or alpha = *alpha_in (device float, nullable; takes precedence,
 * e.g. the output of bhfwi_line_search); then mu is clipped to
 * rho [vs_min^2, vs_max^2] and lam + 2 mu to rho [vp_min^2, vp_max^2].
 * alpha_out (device float, nullable) receives alpha. */
int bhfwi_update(bhfwi_ctx *ctx, void *stream, int64_t n, float *lam, float *mu,
                 const float *rho, const float *g_lam, const float *g_mu, const uint8_t *mask,
                 float eta, float alpha_override, const float *alpha_in,
                 const bhfwi_bounds *bounds, float *alpha_out);

#ifdef __cplusplus
}
#endif
#endif
