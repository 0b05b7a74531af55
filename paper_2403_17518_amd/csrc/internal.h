// Internal declarations shared by the kernels (fwi_kernels.hip) and the
// host planner / C ABI (fwi_api.hip). Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

struct fwi_ctx;

namespace fwi {

constexpr int kLanes = 64;          // wavefront width on CDNA
constexpr int kHalo = 4;            // stencil radius (8th order)
constexpr int kWavesPerBlock = 4;   // waves per workgroup of the step kernels
// A wavefield of one shot is stored as (NZ + 2*kZeroRows + 2) rows of pitch
// P: one guard row, kZeroRows zero rows, NZ padded rows, kZeroRows zero rows,
// one guard row. Columns NX .. P-1 of every row stay zero (P >= NX +
// kZeroRows), so they serve as the right halo of a row and, read through the
// flat index, as the left halo of the next row. Eight zero rows/columns cover
// the reach of two stencil applications (two time levels per launch).
constexpr int kZeroRows = 2 * kHalo;
constexpr int kRowsAbove = kZeroRows + 1;
constexpr int kRowsExtra = 2 * kZeroRows + 2;

// Per-shot layout and acquisition (device table, indexed in "slot" order:
// shots sorted by decreasing record length).
struct ShotDesc {
    int64_t f_off;   // float offset of padded cell (0,0) in a field buffer
    int64_t g_off;   // float offset of padded cell (0,0) in an image / D slot
    int32_t P;       // row pitch (floats)
    int32_t NX;      // padded width = win_nx + 2 nb
    int32_t x0;      // first model column of the window
    int32_t wnx;     // window width
    int32_t nt;      // record length
    int32_t src_i;   // source row, padded coordinates
    int32_t src_j;   // source column, padded coordinates
    int32_t wav_off; // float offset of the shot's wavelet
    // bilinear source weights of cells (src_i + a, src_j + b), index 2a + b
    // (1, 0, 0, 0 for a source on the grid)
    float sw00, sw01, sw10, sw11;
};

// One wavefront of a step kernel owns the columns [col0, col0 + width) and
// the rows [z0, z1) of one shot. Its lanes hold the columns starting at
// col0 (one level per launch, width = 64*cw) or col0 - 4 (two levels per
// launch, width = 64*cw - 8: the outer 4 columns on each side are computed
// at the intermediate level only). Rows holding receivers among the lanes'
// columns are listed in rrows[rr0 .. rr1) (for two levels: rows z0-4 ..
// z1+3).
struct WaveDesc {
    int32_t shot, col0, z0, z1;
    int32_t rr0, rr1, pad0, pad1;
};

// A row of a strip that holds receiver cells: rmap[map_off + lane] is the
// unique-receiver-cell index q of column col0 + lane, or -1.
struct RecRow {
    int32_t row, map_off;
};

enum StepFlags : int {
    F_SRC = 1,     // add the source term w[n]/h^2
    F_SAMPLE = 2,  // record the new field at receiver cells
    F_INJECT = 4,  // add the adjoint source at receiver cells
    F_EMIT = 8,    // store D^n = V^2 dt^2 (L8 u^n + s^n)
    F_IMAGE = 16,  // accumulate G += out * D^n
    F_SCAT = 32,   // scattered field: source (2 dV / V) D^n from the stored background history
                   // (2 dm D^n for a relative perturbation dm)
};

struct StepArgs {
    const ShotDesc *shots;
    const WaveDesc *waves;
    const RecRow *rrows;
    const int32_t *rmap;
    const float *v;      // physical model [nz][nx]
    const float *dv;     // Born perturbation [nz][nx]
    const float *wav;    // wavelets
    int32_t nwaves, nz, nx, nb, NZ;
    int32_t top;               // padded rows above physical row 0 (nb, or 0 under a free surface)
    int32_t fs;                // free surface: row 0 held at zero, odd mirror above it
    int32_t rel;               // Born perturbation given as dV / V (1) or dV (0)
    int32_t cw;                // columns per lane of the wave table (1 or 2)
    int32_t pd;                // one-level kernel: rows prefetched ahead (1 or 2)
    float w1, w2, w3, w4;      // c_k / h^2 (the centre weight is -4 times their sum)
    float dt2;                 // dt^2
    float hs;                  // smax dt / (2 nb^2): sigma dt/2 = hs (dz^2 + dx^2)
    float ih2;                 // 1 / h^2
    int32_t n;                 // time index (of the first level computed)
    int32_t n2;                // time index of the second level (two-level kernels)
    const float *cur;          // field at the current level
    float *prev;               // previous level in, next level out (one level);
                               // previous level in (two levels)
    float *out1, *out2;        // two-level kernels: the two new levels
    const float *cur2;         // second field (Born)
    float *prev2;
    float *dslot;              // D^n slot (F_EMIT writes, F_IMAGE reads)
    float *G;                  // imaging accumulator
    float *samp;               // receiver samples of step n: samp[q]
    const float *inj;          // adjoint sources of step n: inj[q]
    float *samp2;              // ... of the second level
    const float *inj2;
    float *dslot2;
    // perfectly matched layer (pml != 0): edge fields of the field (psx: x
    // edges (i, j+1/2) at column j; psz: z edges (i+1/2, j) at row i) in the
    // field layout, read at level n-1 and written at level n, and those of
    // the second (Born) field; damping d = hd0 m^2 at a position of m half
    // cells into the layer
    int32_t pml;
    float hd0;                 // smax / (4 nb^2)
    float dt;
    float ih;                  // 1 / h
    const float *psx_in, *psz_in;
    float *psx_out, *psz_out;
    const float *psx2_in, *psz2_in;
    float *psx2_out, *psz2_out;
};

// Time-major <-> trace-major conversion, residual and misfit.
//   tm_out[n][q] = sum over receivers r at cell q of
//                  (alpha * tm_in[n][q] + beta * tr_in[r][n])
//   tr_out[r][n] = tm_in[n][q(r)]
//   partials[block] = 1/2 sum over (r, n) of (alpha*tm_in + beta*tr_in)^2
struct TraceArgs {
    int32_t Q;
    int32_t nt_max;
    const int32_t *q_nt;     // [Q] record length of the cell's shot
    const int32_t *q_rptr;   // [Q+1] receivers of cell q: q_roff[q_rptr[q]..]
    const int64_t *q_roff;   // trace offsets (floats) in the packed data
    // off-grid receivers (offgrid != 0): receiver r combines cells
    // r_cq[r_cptr[r] ..] with weights r_cw[..]; q_rw[k] is the weight of
    // the receiver entry q_roff[k]; resid [data] holds the combined traces
    int32_t offgrid;
    int32_t R;
    const int32_t *r_cptr, *r_cq, *r_nt;
    const float *r_cw, *q_rw;
    const int64_t *r_off;
    float *resid;
    int64_t ndata;           // packed data samples
    const float *tm_in;
    float alpha;
    const float *tr_in;
    float beta;
    float *tm_out;
    float *tr_out;
    double *partials;
};

struct FinalArgs {
    const ShotDesc *shots;
    int32_t nshots;
    float *G;           // folded in place
    const float *v;
    int32_t nz, nx, nb, NZ;
    int32_t top;        // padded rows above physical row 0
    int32_t rel;        // 1: image of the relative perturbation (times v)
    float dt2;
    float *img;
};

// context accessors for the other parts of the library (deblur_api.hip)
hipStream_t ctx_stream(const struct ::fwi_ctx *c);
int ctx_device(const struct ::fwi_ctx *c);

hipError_t launch_step(int flags, const StepArgs &a, hipStream_t s);
hipError_t launch_step2(int flags, const StepArgs &a, hipStream_t s);
hipError_t launch_born_step(const StepArgs &a, hipStream_t s);
hipError_t launch_fill(float *p, int64_t n, float val, hipStream_t s);
// y = a x (n floats)
hipError_t launch_scale(const float *x, float a, float *y, int64_t n, hipStream_t s);
hipError_t launch_model_check(const float *v, int64_t n, float *out3, hipStream_t s);
// dout[off[r] + n] = din[off[r] + n] * mute weight of sample n of trace r
// (ntr traces, nt[r] samples, ramp from t0[r] over `taper` seconds)
hipError_t launch_mute(const int64_t *off, const int32_t *nt, const float *t0, int32_t ntr, float dt, float taper,
                       const float *din, float *dout, hipStream_t s);
// y = 4 x - (its four neighbours), zero outside [nz][nx]
hipError_t launch_laplace5(const float *x, int32_t nz, int32_t nx, float *y, hipStream_t s);
// Writes per-block misfit partials when a.partials is set; their count
// goes to *nblocks_out (at most traces_partials_max(Q, nt_max)).
hipError_t launch_traces(const TraceArgs &a, hipStream_t s, int64_t *nblocks_out);
int64_t traces_partials_max(int32_t Q, int32_t nt_max);
hipError_t launch_sum_partials(const double *part, int64_t n, double *out, hipStream_t s);
hipError_t launch_finalize(const FinalArgs &a, int max_nx, hipStream_t s);

}  // namespace fwi
