/*
 * fwi.h - C ABI of the MI355X finite-difference acoustic propagation library
 * (libfwi.so) behind deep-Hessian-deblurred full waveform inversion.
 *
 * Operators (all on one GPU, FP32, hand-written HIP kernels for gfx950):
 *
 *   fwi_forward   d  = F(v)                       paper section 2.1, eq. 1
 *   fwi_gradient  g  = J^T (F(v) - d_obs),        section 2.1 eq. 2 and
 *                 phi = 1/2 ||F(v) - d_obs||^2    section 2.3 eq. 13
 *   born_demig    dd = J dv                       section 2.2, eq. 11-12b
 *   born_mig      img = J^T dd                    section 2.3, eq. 13
 *
 * where J = dF/dv is the exact Jacobian of the discrete forward map, so
 * born_mig(v, born_demig(v, g)) is the doubly migrated image J^T J g of
 * section 2.3 eq. 15. With fwi_grid.relative = 1 every J above is
 * J diag(v), the operator on relative perturbations dv / v of eq. 12.
 *
 * Discretisation (the paper names the finite-difference method but not a
 * scheme; this is the library's definition): constant-density acoustic wave
 * equation in velocity v, 8th-order central Laplacian on a square grid of
 * spacing h, 2nd-order leapfrog in time,
 *     u^{n+1} = a (2 u^n + V^2 dt^2 (L8 u^n + s^n)) - b u^{n-1},
 * with a damping sponge of nb cells on all four sides
 *     sigma = smax (dz^2 + dx^2), dz, dx = depth into the sponge / nb,
 *     smax = 3 v_ref ln(1/R) / (2 nb h), a = 1/(1 + sigma dt/2),
 *     b = (1 - sigma dt/2) a,
 * zero field values outside the padded box, V = the shot window of v
 * edge-replicated into the sponge, a point source s^n = w[n]/h^2 at the
 * source cell and point receivers d[r][n] = u^{n+1}[rz][rx]. Options:
 * sources and receivers between cells (fwi_geom offsets, bilinear
 * weights), a pressure-free top surface instead of the top sponge
 * (fwi_grid.free_surface), a perfectly matched layer instead of the
 * sponge (fwi_grid.pml), the Born operator on relative perturbations
 * (fwi_grid.relative), and the checkpointing of the adjoint sweeps
 * (fwi_grid.ckpt_every, fwi_ctx_set_mem_budget, fwi_ctx_set_ckpt_slots).
 *
 * Memory and ownership
 *   - Every float pointer argument of an operator is a DEVICE pointer that
 *     the caller owns (e.g. from torch), contiguous, row-major:
 *       models / images      [nz][nx], x fastest;
 *       data                 packed traces: shot order, then the shot's
 *                            receiver order, time fastest, nt[s] samples.
 *   - fwi_grid and fwi_geom are HOST structures; their arrays (including
 *     the wavelet) are host memory and are copied during the call.
 *   - Outputs are overwritten, never accumulated; inputs are not modified.
 *   - Scratch (wavefields, checkpoints, the imaging-condition buffers) is
 *     owned by the context and reused across calls.
 *
 * Streams and threads
 *   - Work is enqueued on the context's stream (fwi_ctx_set_stream). Calls
 *     return once the work is enqueued, except that fwi_gradient with a
 *     non-NULL misfit pointer waits for the result, and every call waits
 *     for the model check described under FWI_ECFL.
 *   - A context is not thread-safe: use one context per host thread.
 *
 * Errors: every int-returning function returns FWI_OK (0) or a negative
 * code; fwi_last_error() gives a message. After an error, outputs are
 * unspecified; the context stays usable unless the error was FWI_EHIP.
 */
#ifndef FWI_H
#define FWI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FWI_OK = 0,
    FWI_EINVAL = -1,   /* bad size, position, window or NULL pointer */
    FWI_ENOMEM = -2,   /* device allocation failed */
    FWI_EHIP = -3,     /* HIP runtime error */
    FWI_ECFL = -4,     /* v dt / h above the stability limit */
    FWI_ESTATE = -5,   /* object used in the wrong state */
    FWI_ENOTIMPL = -6
};

typedef struct fwi_ctx fwi_ctx;

typedef struct {
    int32_t nz, nx;     /* physical model rows (depth) and columns */
    int32_t nb;         /* sponge width in cells on all four sides (three under
                           a free surface), >= 0 */
    float h;            /* grid spacing (m); dz == dx */
    float dt;           /* time step (s) */
    int32_t nt_max;     /* longest record; length of a shared wavelet */
    float v_ref;        /* fixed sponge reference velocity (m/s) */
    float R;            /* nominal sponge reflection coefficient, (0, 1) */
    int32_t ckpt_every; /* checkpoint interval (steps) for the adjoint
                           sweeps; 0 = chosen from the memory budget */
    int32_t free_surface; /* 1: the top of the model (physical row 0) is a
                             pressure-free surface - no sponge above it, u = 0
                             on it, odd mirror above it (image method) */
    int32_t relative;   /* perturbation parametrisation of the Born operator
                           (section 2.2, eq. 12: L acts on dm / m_o).
                           0: absolute velocity, J = dF/dv; born_demig takes
                           dv in m/s, and born_mig, fwi_gradient and the
                           pairs return images per m/s.
                           1: relative perturbation dv / v, J_rel = J diag(v);
                           born_demig takes the dimensionless dv / v, and the
                           images are diag(v) J^T (fwi_gradient then returns
                           the gradient with respect to ln v). */
    int32_t pml;        /* 1: the nb padded cells are a perfectly matched
                           layer instead of the sponge (the same damping
                           profile, in the stretched-coordinate equation
                           multiplied by s_x s_z, which keeps the operator
                           symmetric: the adjoint is the same recursion run
                           backward). Two edge fields per propagated field
                           ride along (memory: four more field-sized buffers
                           per field, snapshots twice as large); every
                           tiling takes the layer, two-level ones included
                           (the intermediate level's edge fields stay in
                           registers). */
} fwi_grid;

typedef struct {
    int32_t nshots;
    const int32_t *src_z, *src_x;   /* [nshots] physical cell of the source */
    const int32_t *win_x0, *win_nx; /* [nshots] column window of each shot;
                                       both NULL = the full width */
    const int32_t *nt;              /* [nshots] record length; NULL = nt_max */
    const int64_t *rec_ptr;         /* [nshots+1] receivers of shot s are
                                       rec_ptr[s] .. rec_ptr[s+1]-1 */
    const int32_t *rec_z, *rec_x;   /* physical cells; co-located receivers
                                       are allowed (their traces are equal
                                       and their adjoint sources add) */
    const float *wavelet;           /* host: [nt_max] if wavelet_shared,
                                       else [nshots][nt_max] */
    int32_t wavelet_shared;
    /* Optional off-grid positions (host, NULL = on the grid): fractional
     * offsets in [0, 1) toward +z and +x from (src_z, src_x) [nshots] and
     * from (rec_z, rec_x) [rec_ptr[nshots]]. A source is spread over the
     * four surrounding cells and a receiver combines them with bilinear
     * weights (1-fz)(1-fx), (1-fz)fx, fz(1-fx), fz fx; a nonzero offset
     * needs the next cell inside the model (z + 1 < nz) or the shot's
     * window (x + 1 < win_x0 + win_nx). Both arrays of a pair are given or
     * both are NULL. */
    const float *src_fz, *src_fx;
    const float *rec_fz, *rec_fx;
} fwi_geom;

typedef struct {
    /* filled by the last operator call on the context */
    double cell_updates;      /* padded-cell x step x shot x field updates */
    int64_t stencil_launches; /* launches of the propagation kernels */
    int32_t ckpt_every;       /* checkpoint interval used (0 = none) */
    int32_t n_segments;       /* adjoint segments (recompute passes + 1) */
    int64_t scratch_bytes;    /* device scratch held by the context */
    /* kernel timings, valid only when profiling is enabled (ms, summed
       over runs of consecutive launches of one class) */
    double ms_fwd, ms_adj, ms_born, ms_other;
    int64_t n_fwd, n_adj, n_born;
    double bytes_fwd, bytes_adj, bytes_born; /* algorithmic bytes moved */
    /* tiling used by the forward, adjoint and Born kernels: columns per
       lane (strip width 64 * cols), rows streamed per wave and time levels
       advanced per launch */
    /* tilings by class: forward, adjoint, joint Born, scattered field */
    int32_t tile_cw[4], tile_rows[4], tile_levels[4];
    int32_t tile_prefetch[4]; /* rows of loads issued ahead */
    int64_t graph_launches;   /* time loops replayed from a captured HIP graph */
    int64_t graph_captures;   /* time loops captured (first run of a loop) */
    int64_t recomputed_steps; /* forward time steps recomputed by the adjoint
                                 sweeps from snapshots */
    int32_t ckpt_slots;       /* snapshots of (u^{n-1}, u^n) the adjoint
                                 sweeps held */
} fwi_stats;

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the default stream). */
int fwi_ctx_create(int device, void *hip_stream, fwi_ctx **out);
void fwi_ctx_destroy(fwi_ctx *ctx);
int fwi_ctx_set_stream(fwi_ctx *ctx, void *hip_stream);
/* Upper bound on device memory used for checkpoints and the stored
 * imaging-condition history (bytes); 0 = 70% of the device memory. The
 * adjoint sweeps store D^n for every step when it fits (no recompute) and
 * otherwise checkpoint; they never plan beyond the memory free at the call
 * minus a 4 GiB margin. */
int fwi_ctx_set_mem_budget(fwi_ctx *ctx, int64_t bytes);
/* Checkpointing of the adjoint sweeps. When the history does not fit, the
 * record is cut into segments of k steps (fwi_grid.ckpt_every, or chosen
 * from the budget) whose D^n history is recomputed, last segment first, from
 * snapshots of (u^{n-1}, u^n) placed by the binomial rule of Griewank's
 * revolve (Griewank & Walther, ACM TOMS 26, 2000): with nseg - 2 snapshots
 * every segment but the last is recomputed once; with fewer, segments are
 * recomputed more often, the fewest times any placement allows. The budget
 * decides the snapshot count (it takes the uniform schedule whenever that
 * fits, else the segment length and snapshot count with the fewest
 * recomputed steps). slots >= 0 caps the count at `slots` (tests, memory
 * held back for other work); -1 (default) removes the cap. Results are the
 * same bits whatever the schedule. */
int fwi_ctx_set_ckpt_slots(fwi_ctx *ctx, int32_t slots);
/* Host only, no device or context needed: replays the schedule the adjoint
 * sweeps follow for nseg segments and `slots` snapshot slots, checking that
 * every recomputation starts from a snapshot of the right segment, that the
 * adjoint takes each segment's freshly recomputed history once, last
 * segment first, and nothing else. *recomputed (nullable) receives the
 * number of segments recomputed. Returns FWI_OK; FWI_EINVAL if nseg < 1 or
 * slots < 0; FWI_ESTATE if a step is out of order (a library bug). */
int fwi_checkpoint_schedule(int32_t nseg, int32_t slots, int64_t *recomputed);
/* 1 = time the propagation kernels with HIP events recorded around every
 * run of consecutive launches of one kernel class (forward, adjoint, Born),
 * so the reported per-launch time includes the (small) gaps between
 * back-to-back launches; adds a stream sync at the end of each call. */
int fwi_ctx_set_profiling(fwi_ctx *ctx, int enable);
/* Tiling of the step kernels. kernel: 0 forward, 1 adjoint, 2 joint Born,
 * 3 scattered field driven by a stored history (fwi_gradient_pair), -1 all;
 * cols_per_lane 1 or 2, rows_per_wave >= 1, levels_per_launch 1 or 2 (the
 * joint Born kernel always advances one level and prefetches one row;
 * levels 2 for it alone is FWI_EINVAL) and prefetch_rows 1 or 2 (rows of loads
 * issued ahead; 0 = 2 for one level, 1 for two) force a tiling; all zero
 * returns the kernel to the autotuner. Results do not depend on the tiling:
 * every variant computes each cell with the same arithmetic. */
int fwi_ctx_set_tiling(fwi_ctx *ctx, int kernel, int cols_per_lane, int rows_per_wave,
                       int levels_per_launch, int prefetch_rows);
/* 1 (default): pick each kernel's tiling by timing candidates once per
 * geometry; 0: use a fixed default tiling. */
int fwi_ctx_set_autotune(fwi_ctx *ctx, int enable);
/* 1 (default): every time loop (a forward, adjoint or Born sweep over a
 * range of steps) is captured once into a HIP graph and replayed on later
 * calls with the same geometry, tiling and scratch buffers; the loops read
 * only context-owned memory (the model and perturbation are copied in at
 * the start of a call), so a graph stays valid across calls whatever
 * buffers the caller passes. 0: launch every step directly. Results are
 * identical either way. */
int fwi_ctx_set_graphs(fwi_ctx *ctx, int enable);
int fwi_ctx_get_stats(const fwi_ctx *ctx, fwi_stats *out);
/* Release all scratch memory and captured graphs held by the context. */
int fwi_ctx_trim(fwi_ctx *ctx);
const char *fwi_last_error(const fwi_ctx *ctx);

/* d = F(v). v: [nz][nx] velocities (m/s); d: packed traces. */
int fwi_forward(fwi_ctx *ctx, const fwi_grid *grid, const fwi_geom *geom,
                const float *v, float *d);

/* d = F(v) as fwi_forward computes it (the same kernels: the same bits),
 * for callers that cannot allocate device memory (serving loops and
 * harnesses that forbid hipMalloc): the call allocates nothing. Its scratch
 * (the plan tables, the two wavefield levels, the receiver samples and the
 * model copy) comes from a static device array of 64 MiB that each device
 * the library runs on holds until the process ends; a problem that needs
 * more returns FWI_ENOMEM (with the size in fwi_last_error) before any
 * propagation runs. The context's own buffers, plan, tilings and captured
 * loops are neither used nor changed; the tiling is the forced one
 * (fwi_ctx_set_tiling) or the fixed default, never autotuned, and no loop is
 * captured. Every allocation-free call on a device shares that device's
 * array and leaves its contents behind: such calls that overlap on one
 * device (other streams, other contexts, other host threads) race. Waits
 * for the model check, as every operator does. */
int fwi_forward_noalloc(fwi_ctx *ctx, const fwi_grid *grid, const fwi_geom *geom,
                        const float *v, float *d);

/* g = J^T (F(v) - d_obs), the gradient of phi = 1/2 ||F(v) - d_obs||^2
 * with respect to v (the negative of the paper's g = L^T (d_o - d_s)).
 * misfit: HOST pointer, may be NULL (then the call does not wait);
 * d_syn: device [packed data] receives F(v), may be NULL. */
int fwi_gradient(fwi_ctx *ctx, const fwi_grid *grid, const fwi_geom *geom,
                 const float *v, const float *d_obs, float *g,
                 double *misfit, float *d_syn);

/* misfit = 1/2 ||F(v) - d_obs||^2 (section 2.1 eq. 2) without the adjoint:
 * one forward sweep and the residual reduction (line searches). misfit is a
 * HOST pointer; the call waits for it. */
int fwi_misfit(fwi_ctx *ctx, const fwi_grid *grid, const fwi_geom *geom,
               const float *v, const float *d_obs, double *misfit);

/* dd = J dv: Born (single-scattering) data of the perturbation dv of the
 * background velocity v0. */
int born_demig(fwi_ctx *ctx, const fwi_grid *grid, const fwi_geom *geom,
               const float *v0, const float *dv, float *dd);

/* img = J^T dd: migration of data dd in the background v0 (the adjoint of
 * born_demig; shot images are summed). */
int born_mig(fwi_ctx *ctx, const fwi_grid *grid, const fwi_geom *geom,
             const float *v0, const float *dd, float *img);

/* RTM image of observed data in the model v, the image product with which
 * the paper compares inverted models (section 3.3): img = Lap5(J^T (M
 * d_obs)), where M mutes the direct arrival and Lap5 y = 4 y - (its four
 * neighbours), zero outside [nz][nx], suppresses the low-wavenumber
 * backscatter of the cross-correlation image. The mute weights sample n
 * (time n dt) of the trace of receiver r by 0 up to t0 = |x_r - x_s| h /
 * mute_v + mute_pad (positions with their off-grid offsets), then by a
 * half-cosine ramp over mute_taper seconds, then by 1; mute_v = 0 skips it.
 * v, img: device [nz][nx]; d_obs: device packed traces. FWI_EINVAL for a
 * negative or non-finite mute velocity or taper. */
int fwi_rtm(fwi_ctx *ctx, const fwi_grid *grid, const fwi_geom *geom, const float *v, const float *d_obs,
            float mute_v, float mute_pad, float mute_taper, float *img);

/* img = J^T J dv, the doubly migrated image of section 2.3 eq. 15 (the
 * Gauss-Newton Hessian applied to dv), and optionally dd = J dv (NULL to
 * skip). One joint Born sweep supplies both the data and the background
 * wavefield of the migration, so the result equals
 * born_mig(v0, born_demig(v0, dv)) bit for bit with one background sweep
 * fewer. v0, dv, img: device [nz][nx]; dd: device packed traces. */
int born_pair(fwi_ctx *ctx, const fwi_grid *grid, const fwi_geom *geom,
              const float *v0, const float *dv, float *dd, float *img);

/* The gradient and its doubly migrated image at the same model, as one FWI
 * iteration of the network method needs them (section 2.3 eq. 13 and 15):
 * grad = J^T (F(v) - d_obs) (as fwi_gradient, bit for bit), misfit (host,
 * nullable), img = J^T J (scale * grad) and, if dd is not NULL, the
 * demigrated data dd = J (scale * grad) (device, packed traces). When the
 * forward sweep's imaging history fits in memory whole (no checkpoints),
 * the pair reuses it: only the scattered field is propagated, with the
 * source (2 dV / V) D^n read from the stored background history, then the
 * adjoint. Otherwise the pair runs as born_pair (and dd, img equal
 * born_pair(v, scale * grad) bit for bit). In the stored-history case dd
 * and img equal born_pair's up to FP32 rounding (the scattered source is
 * formed from the stored D^n). */
int fwi_gradient_pair(fwi_ctx *ctx, const fwi_grid *grid, const fwi_geom *geom,
                      const float *v, const float *d_obs, float *grad, double *misfit,
                      float scale, float *img, float *dd);

#ifdef __cplusplus
}
#endif

#endif /* FWI_H */
