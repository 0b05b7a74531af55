// HIP kernels (gfx950) of the finite-difference acoustic propagation path.
//
// Step kernels: one launch advances every active shot by one time level of
//     u^{n+1} = a (2 u^n + V^2 dt^2 (L8 u^n + s^n)) - b u^{n-1}
// (paper section 2.1 eq. 1, discretised with an 8th-order Laplacian and
// leapfrog time stepping; a, b are the sponge coefficients). The same update
// run backward in time with the receiver residual as source is the adjoint
// (section 2.3 eq. 13), and the two-field variant is the jointly solved Born
// system of section 2.2 eq. 9-11.
//
// Work decomposition: a wavefront owns a strip of 64*CW columns of one shot
// (CW = 1 or 2 columns per lane) and a run of rows. It streams down z keeping
// the nine rows of the current field that the vertical stencil needs in
// registers; the horizontal neighbours of the centre row go through an LDS
// row (the strip plus two 4-cell halos). The kernel is bound by HBM/MALL
// bandwidth (about 1.7 flop per byte), so no matrix cores are involved.
#include <algorithm>

#include "internal.h"

namespace fwi {
namespace {

__device__ __forceinline__ void wave_sync()
{
    // Orders the wave's own LDS traffic: lanes exchange data through LDS
    // without a workgroup barrier (each wave of a block is independent).
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int clampi(int v, int lo, int hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

// Workgroups are dealt round-robin to the 8 XCDs. Remap so that each XCD
// receives a contiguous range of work items: neighbouring strips and rows of
// one shot then share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nblocks)
{
    const int per = nblocks / 8, rem = nblocks % 8;
    const int x = b % 8, k = b / 8;
    return x * per + min(x, rem) + k;
}

// Receiver-row cursor value once a wave's list of receiver rows is used up.
// It must never equal a row index: the two-level kernel walks rows from 4
// (level 1) and 8 (level 2) above the padded box, so -1 is a real row there.
constexpr int kNoRow = -(1 << 30);

// Source weights of a lane's columns: a source off the grid is spread over
// the cells (src_i + a, src_j + b), a, b in {0, 1}, with bilinear weights
// (on the grid: 1 at the source cell, 0 elsewhere, and the fused add below
// is the plain add). w0[k] / w1[k] hold the weights of column k on rows
// src_i / src_i + 1 (zero off the source columns); src_k = src_j - j0.
template <int CW>
__device__ __forceinline__ void source_weights(const ShotDesc &S, int src_k, float (&w0)[CW], float (&w1)[CW])
{
#pragma unroll
    for (int k = 0; k < CW; ++k) {
        const int b = k - src_k;
        w0[k] = b == 0 ? S.sw00 : (b == 1 ? S.sw01 : 0.0f);
        w1[k] = b == 0 ? S.sw10 : (b == 1 ? S.sw11 : 0.0f);
    }
}

// the source term on row r (wave-uniform) of column k
template <int CW>
__device__ __forceinline__ float add_source(float lap, float wsrc, int r, int src_i, const float (&w0)[CW],
                                            const float (&w1)[CW], int k)
{
    if (r == src_i) return __builtin_fmaf(wsrc, w0[k], lap);
    if (r == src_i + 1) return __builtin_fmaf(wsrc, w1[k], lap);
    return lap;
}

__device__ __forceinline__ float sponge_a(float sh)
{
    return __builtin_amdgcn_rcpf(1.0f + sh);
}

// 8th-order Laplacian at column k of a lane's strip: the column's rows
// z-4..z+4 sit in q[0..8][k], the row's columns x-4..x+4 in xr[k..k+8].
// Every neighbour enters as its difference to the centre value (the weights
// sum to zero), so a smooth field loses no significant bits to the large
// centre weight; the smallest weights are summed first.
template <int CW>
__device__ __forceinline__ float lap8(const float (&q)[9][CW], const float *xr, int k,
                                      float w1, float w2, float w3, float w4)
{
    const float c = q[4][k];
    float s = w4 * (((q[0][k] - c) + (q[8][k] - c)) + ((xr[k] - c) + (xr[k + 8] - c)));
    s = __builtin_fmaf(w3, ((q[1][k] - c) + (q[7][k] - c)) + ((xr[k + 1] - c) + (xr[k + 7] - c)), s);
    s = __builtin_fmaf(w2, ((q[2][k] - c) + (q[6][k] - c)) + ((xr[k + 2] - c) + (xr[k + 6] - c)), s);
    s = __builtin_fmaf(w1, ((q[3][k] - c) + (q[5][k] - c)) + ((xr[k + 3] - c) + (xr[k + 5] - c)), s);
    return s;
}

// Leapfrog update with the sponge, a (2u + D) - b u_prev where a = 1/(1+sh)
// and b = (1-sh) a, written as a ((u - u_prev) + u + D + sh u_prev): the
// change over one step is formed first, which keeps the low bits of a slowly
// varying field (a = 1, sh = 0 away from the sponge).
__device__ __forceinline__ float leapfrog(float u, float up, float D, float a, float sh)
{
    return a * (((u - up) + u) + __builtin_fmaf(sh, up, D));
}

template <int CW>
__device__ __forceinline__ void ld(const float *p, float (&o)[CW])
{
    if constexpr (CW == 1) {
        o[0] = *p;
    } else {
        const float2 t = *reinterpret_cast<const float2 *>(p);
        o[0] = t.x;
        o[1] = t.y;
    }
}

// Raw buffer view of a wave-uniform base address. A load or store names the
// base by its descriptor (scalar registers), a per-row byte offset (scalar)
// and a fixed per-lane byte offset (one vector register), so streaming a row
// costs no vector address arithmetic. Range checking is left wide open:
// every offset used is in bounds by construction, except on purpose: a load
// whose lane offset lies past the range (kNoLoad) returns zeros without a
// memory request, and such a store is dropped. Loads that a lane or a row
// does not need are made that way instead of being skipped, so that no load
// sits in a branch; the step kernels store their columns that way too (lanes
// past the shot's width, columns a two-level wave does not own), without a
// per-lane branch. The loads and stores are the
// raw-buffer intrinsics of the AMDGPU backend, bound by name.
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ float raw_ld_f32(i32x4 rsrc, int voff, int soff, int aux) __asm("llvm.amdgcn.raw.buffer.load.f32");
__device__ f32x2 raw_ld_v2f32(i32x4 rsrc, int voff, int soff, int aux) __asm("llvm.amdgcn.raw.buffer.load.v2f32");
__device__ f32x4 raw_ld_v4f32(i32x4 rsrc, int voff, int soff, int aux) __asm("llvm.amdgcn.raw.buffer.load.v4f32");
__device__ void raw_st_f32(float v, i32x4 rsrc, int voff, int soff, int aux) __asm("llvm.amdgcn.raw.buffer.store.f32");
__device__ void raw_st_v2f32(f32x2 v, i32x4 rsrc, int voff, int soff, int aux) __asm("llvm.amdgcn.raw.buffer.store.v2f32");

using Rsrc = i32x4;
constexpr int kRsrcWord3 = 0x00020000;   // 32-bit data format, no swizzle

__device__ __forceinline__ Rsrc view(const float *base)
{
    const unsigned long long a = reinterpret_cast<unsigned long long>(base);
    Rsrc r;
    r.x = int(unsigned(a));
    r.y = int(unsigned(a >> 32) & 0xffffu);   // stride 0
    r.z = 0x7fffffff;                        // byte range
    r.w = kRsrcWord3;
    return r;
}

constexpr unsigned kNoLoad = 0x80000000u;   // a lane offset past every view's range

__device__ __forceinline__ float bld1(Rsrc r, unsigned lane_off, int row_off)
{
    return raw_ld_f32(r, int(lane_off), row_off, 0);
}

template <int CW>
__device__ __forceinline__ void bld(Rsrc r, unsigned lane_off, int row_off, float (&o)[CW])
{
    if constexpr (CW == 1) {
        o[0] = bld1(r, lane_off, row_off);
    } else {
        const f32x2 t = raw_ld_v2f32(r, int(lane_off), row_off, 0);
        o[0] = t.x;
        o[1] = t.y;
    }
}

__device__ __forceinline__ float4 bld4(Rsrc r, unsigned lane_off, int row_off)
{
    const f32x4 t = raw_ld_v4f32(r, int(lane_off), row_off, 0);
    return make_float4(t.x, t.y, t.z, t.w);
}

__device__ __forceinline__ void bst1(Rsrc r, unsigned lane_off, int row_off, float v)
{
    raw_st_f32(v, r, int(lane_off), row_off, 0);
}

// The D^n history is written once per step and read once, much later, by
// another sweep: its loads and stores carry the non-temporal cache policy
// (bit 1 of the cache-policy operand) so that the stream does not displace
// the fields and the image accumulator, which are re-read every step.
constexpr int kStream = 2;

template <int CW>
__device__ __forceinline__ void bld_stream(Rsrc r, unsigned lane_off, int row_off, float (&o)[CW])
{
    if constexpr (CW == 1) {
        o[0] = raw_ld_f32(r, int(lane_off), row_off, kStream);
    } else {
        const f32x2 t = raw_ld_v2f32(r, int(lane_off), row_off, kStream);
        o[0] = t.x;
        o[1] = t.y;
    }
}

// A lane's CW values of one row of the history; ok[k] marks the columns it
// owns (ok[1] implies ok[0]). Two columns go out as one 8-byte store: two
// 4-byte non-temporal stores from every lane would leave each cache line
// written in halves.
template <int CW>
__device__ __forceinline__ void bst_stream(Rsrc r, unsigned lane_off, int row_off, const float (&v)[CW],
                                           const bool (&ok)[CW])
{
    if constexpr (CW == 2) {
        if (ok[1]) {
            f32x2 t;
            t.x = v[0];
            t.y = v[1];
            raw_st_v2f32(t, r, int(lane_off), row_off, kStream);
            return;
        }
    }
    if (ok[0]) raw_st_f32(v[0], r, int(lane_off), row_off, kStream);
}

// ---- perfectly matched layer ---------------------------------------------
// The layer adds to the Laplacian the divergence of two edge fields: psi_x on
// the x edges (i, j+1/2), stored at column j, and psi_z on the z edges
// (i+1/2, j), stored at row i, each advanced from its previous level by the
// recursive convolution psi^n = b psi^{n-1} + (e - d) g (u^n across the edge)
// / h, where d is the damping along the edge's own axis (at the edge), e the
// damping along the other axis (at the edge's row or column), b = exp(-d dt),
// g = (1 - b) / d (dt where d = 0); and -d_x d_z dt^2 u^n to the update. A
// wave computes the edges it owns (the right and lower edge of each cell)
// and recomputes, from the previous level, the edge left of its strip and the
// edge above its first row, which neighbouring waves own: every edge value is
// formed from the same operands in the same order whichever wave forms it.

// Squared depth into the layer, in half cells, of the position m half cells
// along an axis of n cells with a layer of lo cells at the low end and nb at
// the high end; the damping there is smax (depth / nb)^2 = hd0 * m2 with
// hd0 = smax / (4 nb^2). Dampings are formed from these integers, and the
// difference of two dampings as hd0 * (m2 - m2'), exactly: a difference of
// two rounded products would leave the compiler free to fuse one of them
// into the subtraction, which rounds differently where both are non-zero
// (the corners), and differently in different kernels.
__device__ __forceinline__ int pml_m2(int m, int n, int lo, int nb)
{
    const int d = max(max(2 * lo - m, m - 2 * (n - 1 - nb)), 0);
    return d * d;
}

__device__ __forceinline__ void pml_rec(float d, float dt, float &b, float &g)
{
    b = expf(-d * dt);
    g = d > 0.f ? -expm1f(-d * dt) / d : dt;
}

// new value of an edge from its previous value; ed = e - d, du = u(after) -
// u(before) across the edge
__device__ __forceinline__ float pml_edge(float old, float b, float g, float ed, float du, float ih)
{
    return __builtin_fmaf(b, old, (ed * g) * (du * ih));
}

// Per-lane layer coefficients of a strip's columns: damping of the column
// (cell) and of its right edge with that edge's recursion, and the recursion
// of the edge left of the lane's first column.
template <int CW>
struct PmlCols {
    int mxc[CW], mxe[CW], mxl;  // squared half-cell depths: column, right edge, left edge
    float dxc[CW], bxe[CW], gxe[CW];
    bool xok[CW];               // the column and its right edge lie inside the box
    float bxl, gxl;
    bool lok;                   // the left edge lies inside the box
    __device__ __forceinline__ void init(const StepArgs &A, int j0, int NX)
    {
#pragma unroll
        for (int k = 0; k < CW; ++k) {
            const int j = j0 + k;
            mxc[k] = pml_m2(2 * j, NX, A.nb, A.nb);
            mxe[k] = pml_m2(2 * j + 1, NX, A.nb, A.nb);
            dxc[k] = A.hd0 * float(mxc[k]);
            pml_rec(A.hd0 * float(mxe[k]), A.dt, bxe[k], gxe[k]);
            xok[k] = j >= 0 && j + 1 < NX;
        }
        mxl = pml_m2(2 * j0 - 1, NX, A.nb, A.nb);
        pml_rec(A.hd0 * float(mxl), A.dt, bxl, gxl);
        lok = j0 >= 1;
    }
};

// Per-row layer coefficients: depth and damping of row z (cell), depth of
// the edge below it and that edge's recursion.
struct PmlRow {
    int mzc, mze;
    float dzc, bze, gze;
    bool zok;                   // the edge below lies inside the box
    __device__ __forceinline__ void init(const StepArgs &A, int z)
    {
        mzc = pml_m2(2 * z, A.NZ, A.top, A.nb);
        mze = pml_m2(2 * z + 1, A.NZ, A.top, A.nb);
        dzc = A.hd0 * float(mzc);
        pml_rec(A.hd0 * float(mze), A.dt, bze, gze);
        zok = z >= 0 && z + 1 < A.NZ;
    }
};

// Rows whose cells read a non-zero edge field in a strip without layer
// columns: the layer rows and the first row below / last row above them.
__device__ __forceinline__ bool pml_row(const StepArgs &A, int z)
{
    return z <= A.top || z >= A.NZ - 1 - A.nb;
}

// Strips whose columns reach the layer or the column next to it.
template <int CW>
__device__ __forceinline__ bool pml_strip(const StepArgs &A, int col0, int NX)
{
    return col0 <= A.nb || col0 + kLanes * CW - 1 >= NX - 1 - A.nb;
}

// One row of the layer terms of a field: new edge values from the previous
// ones (own right and lower edges; for lane 0 the edge left of the strip;
// the edge above comes from `up`, the previous row's lower edges), and
// div[k], the edge differences that divided by h give the divergence (the
// caller adds div * (1/h) to the Laplacian as one fused multiply-add, so that
// every kernel rounds it alike); up[] becomes this row's lower edges.
template <int CW>
__device__ __forceinline__ void pml_row_terms(const StepArgs &A, const PmlCols<CW> &C, const PmlRow &R, int lane,
                                              const float (&q)[9][CW], const float *xr, const float (&px)[CW],
                                              const float (&pz)[CW], float pxl, float (&nx)[CW], float (&nz)[CW],
                                              float (&up)[CW], float (&div)[CW])
{
    const float ih = A.ih;
#pragma unroll
    for (int k = 0; k < CW; ++k) {
        const float c = q[4][k];
        // x edge: e = d_z of the row, d = d_x of the edge; z edge: e = d_x of
        // the column, d = d_z of the edge
        nx[k] = C.xok[k] ? pml_edge(px[k], C.bxe[k], C.gxe[k], A.hd0 * float(R.mzc - C.mxe[k]), xr[k + 5] - c, ih)
                         : 0.f;
        nz[k] = R.zok ? pml_edge(pz[k], R.bze, R.gze, A.hd0 * float(C.mxc[k] - R.mze), q[5][k] - c, ih) : 0.f;
    }
    // the edge left of each column: the previous column's right edge, for
    // the lane's first column from the lane to the left, for lane 0 formed
    // here from the previous level
    float left = __shfl_up(nx[CW - 1], 1, kLanes);
    if (lane == 0)
        left = C.lok ? pml_edge(pxl, C.bxl, C.gxl, A.hd0 * float(R.mzc - C.mxl), q[4][0] - xr[3], ih) : 0.f;
#pragma unroll
    for (int k = 0; k < CW; ++k) {
        const float l = k == 0 ? left : nx[k - 1];
        div[k] = (nx[k] - l) + (nz[k] - up[k]);
        up[k] = nz[k];
    }
}

// Receiver rows. The entries of a wave's row list are wave-uniform: read
// through the constant address space they become scalar loads, which the
// vector-memory counter does not track. The per-lane receiver indices (and
// the adjoint's injected values) are vector loads made on receiver rows only;
// the wave waits for them there, so that on every other row the compiler has
// no outstanding load of unknown position to wait for and the row prefetch
// stays in flight.
typedef const __attribute__((address_space(4))) RecRow *RecRowsK;
__device__ __forceinline__ RecRowsK rec_rows(const RecRow *p) { return (RecRowsK)p; }
__device__ __forceinline__ void vm_drain() { __builtin_amdgcn_s_waitcnt(0x0F70); }   // vmcnt(0)

template <int CW, bool INJ>
__device__ __forceinline__ void receiver_row(const StepArgs &A, RecRowsK rrows, const float *inj, int &rr,
                                             int &rrow, int rr_end, int lane, int (&qi)[CW], float (&iv)[CW])
{
    const int mo = rrows[rr].map_off + CW * lane;
#pragma unroll
    for (int k = 0; k < CW; ++k) qi[k] = A.rmap[mo + k];
    if (INJ) {
#pragma unroll
        for (int k = 0; k < CW; ++k) iv[k] = qi[k] >= 0 ? inj[qi[k]] : 0.f;
    }
    ++rr;
    rrow = rr < rr_end ? rrows[rr].row : kNoRow;
    vm_drain();
}

// One time level of every active shot. Each lane owns CW adjacent columns of
// a 64*CW-column strip and streams down the rows [z0, z1) of that strip; the
// loads of rows z+1 .. z+PD are issued before row z is computed so that PD+1
// rows of memory traffic are in flight per wave.
template <int FL, int CW, int PD, bool PML>
__global__ __launch_bounds__(kLanes *kWavesPerBlock) void k_step(const StepArgs A)
{
    constexpr int SW = kLanes * CW;          // strip width
    constexpr int RW = SW + 2 * kHalo;       // LDS row width
    __shared__ float lds[kWavesPerBlock][RW];
    const int lane = threadIdx.x & (kLanes - 1);
    // wave-uniform from here on: descriptors, bases and row offsets live in
    // scalar registers
    const int wl = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    const int wid = xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wl;
    if (wid >= A.nwaves) return;  // whole wave leaves; no block barrier used
    float *row = lds[wl];
    const WaveDesc W = A.waves[wid];
    const ShotDesc S = A.shots[W.shot];
    const int P = S.P;
    const int nb = A.nb;
    const int j0 = W.col0 + CW * lane;       // first column of this lane
    // every load is unconditional: lanes past the shot's width read a zero
    // column (P - CW >= NX + 2) instead
    const unsigned jl = 4u * unsigned(min(j0, P - 2));   // byte offsets
    const unsigned js = 4u * unsigned(j0);
    // offsets below are relative to the field block start (guard row), so
    // they are non-negative 32-bit values
    const float *cu = A.cur + (S.f_off - int64_t(kRowsAbove) * P);
    float *pv = A.prev + (S.f_off - int64_t(kRowsAbove) * P);
    const Rsrc rcur = view(cu), rprev = view(pv), rv = view(A.v);
    const Rsrc rg = view((FL & F_IMAGE) ? A.G + S.g_off : A.v);
    const Rsrc rd = view((FL & (F_IMAGE | F_EMIT | F_SCAT)) ? A.dslot + S.g_off : A.v);
    const Rsrc rdv = view((FL & F_SCAT) ? A.dv : A.v);

    bool valid[CW];
    unsigned jm[CW], jsv[CW];
    float dx2[CW], ax[CW], shx[CW];
#pragma unroll
    for (int k = 0; k < CW; ++k) {
        const int j = j0 + k;
        valid[k] = j < S.NX;
        // store offset of the column: past the range (stores dropped) when the
        // column lies past the shot's width, so that no store sits in a branch
        jsv[k] = valid[k] ? 4u * unsigned(j) : kNoLoad;
        jm[k] = 4u * unsigned(S.x0 + clampi(j - nb, 0, S.wnx - 1));
        const int ddx = max(max(nb - j, j - (S.NX - 1 - nb)), 0);
        dx2[k] = float(ddx * ddx);
        const float sh = A.hs * dx2[k];
        ax[k] = sponge_a(sh);
        shx[k] = sh;
    }
    // halo: lane 0 reads the 4 columns left of the strip, lane 1 the 4
    // columns right of it (a zero column block when past the shot's width)
    // (byte offset shifted up by the 4 halo columns so that it is never
    // negative; the row offset of the load is lowered by as much)
    const unsigned hcol =
        lane < 2 ? 4u * unsigned(lane == 0 ? W.col0 : min(W.col0 + SW, P - kHalo) + kHalo) : kNoLoad;

    // perfectly matched layer: edge fields in the field layout
    PmlCols<CW> pc;
    bool pstrip = false;
    Rsrc rpxi = rv, rpzi = rv, rpxo = rv, rpzo = rv;
    float pup[CW], pup_old[CW];
    const unsigned jleft = 4u * unsigned(max(W.col0 - 1, 0));
    if constexpr (PML) {
        pc.init(A, j0, S.NX);
        pstrip = pml_strip<CW>(A, W.col0, S.NX);
        const int64_t fb = S.f_off - int64_t(kRowsAbove) * P;
        rpxi = view(A.psx_in + fb);
        rpzi = view(A.psz_in + fb);
        rpxo = view(A.psx_out + fb);
        rpzo = view(A.psz_out + fb);
#pragma unroll
        for (int k = 0; k < CW; ++k) pup[k] = pup_old[k] = 0.f;
        // the edges above the first row, owned by the wave above
        if ((pstrip || pml_row(A, W.z0)) && W.z0 >= 1) bld<CW>(rpzi, jl, 4 * (W.z0 - 1 + kRowsAbove) * P, pup_old);
    }

    float q[9][CW];
#pragma unroll
    for (int r = 0; r < 8; ++r) bld<CW>(rcur, jl, 4 * (W.z0 - kHalo + r + kRowsAbove) * P, q[r]);

    // prefetched loads of one row; PD rows are in flight ahead of the row
    // being computed (a ring of PD statically indexed slots)
    struct Pre {
        float q[CW], pv[CW], v[CW], d[CW], g[CW], dv[CW];
        float px[CW], pz[CW], pxl;
        float4 h;
    };
    auto prefetch = [&](int z, Pre &pre) {
        const int ro = 4 * (z + kRowsAbove) * P;
        bld<CW>(rcur, jl, ro + 4 * kHalo * P, pre.q);
        bld<CW>(rprev, jl, ro, pre.pv);
        // lanes 0 and 1 read the halo columns; the other lanes' loads return
        // zeros (kNoLoad), so that no load of the row sits in a branch and
        // the compiler knows how many are in flight
        pre.h = bld4(rcur, hcol, ro - 4 * kHalo);
        const int vo = 4 * clampi(z - A.top, 0, A.nz - 1) * A.nx;
#pragma unroll
        for (int k = 0; k < CW; ++k) pre.v[k] = bld1(rv, jm[k], vo);
        if (FL & F_IMAGE) {
            bld_stream<CW>(rd, jl, 4 * z * P, pre.d);
            bld<CW>(rg, jl, 4 * z * P, pre.g);
        }
        if (FL & F_SCAT) {
            bld_stream<CW>(rd, jl, 4 * z * P, pre.d);
#pragma unroll
            for (int k = 0; k < CW; ++k) pre.dv[k] = bld1(rdv, jm[k], vo);
        }
        if constexpr (PML) {
            if (pstrip || pml_row(A, z)) {
                bld<CW>(rpxi, jl, ro, pre.px);
                bld<CW>(rpzi, jl, ro, pre.pz);
                pre.pxl = lane == 0 ? bld1(rpxi, jleft, ro) : 0.f;
            }
        }
    };

    const RecRowsK rrows = rec_rows(A.rrows);
    int rr = W.rr0;
    int rrow = kNoRow;
    if (FL & (F_SAMPLE | F_INJECT)) rrow = rr < W.rr1 ? rrows[rr].row : kNoRow;
    const float wsrc = (FL & F_SRC) ? A.wav[S.wav_off + A.n] * A.ih2 : 0.0f;
    const int src_k = S.src_j - j0;          // column of the source in this lane, if 0..CW-1
    float sw0[CW], sw1[CW];
    if (FL & F_SRC) source_weights<CW>(S, src_k, sw0, sw1);

    auto do_row = [&](int z, const Pre &c) {
#pragma unroll
        for (int k = 0; k < CW; ++k) q[8][k] = c.q[k];
        // centre row into LDS, then the horizontal neighbours back out
        if constexpr (CW == 1) row[kHalo + lane] = q[4][0];
        else *reinterpret_cast<float2 *>(&row[kHalo + CW * lane]) = make_float2(q[4][0], q[4][1]);
        if (lane < 2) *reinterpret_cast<float4 *>(&row[lane == 0 ? 0 : kHalo + SW]) = c.h;
        wave_sync();
        float xr[CW + 2 * kHalo];
#pragma unroll
        for (int m = 0; m < CW + 2 * kHalo; ++m) xr[m] = row[CW * lane + m];
        wave_sync();

        int qi[CW];
        float iv[CW];
#pragma unroll
        for (int k = 0; k < CW; ++k) {
            qi[k] = -1;
            iv[k] = 0.f;
        }
        if (FL & (F_SAMPLE | F_INJECT))
            if (z == rrow) receiver_row<CW, (FL & F_INJECT) != 0>(A, rrows, A.inj, rr, rrow, W.rr1, lane, qi, iv);
        const int ddz = max(max(A.top - z, z - (A.NZ - 1 - nb)), 0);
        const float dz2 = float(ddz * ddz);
        // layer terms of this row: edge divergence and d_x d_z dt^2
        float pdiv[CW], pnx[CW], pnz[CW], fdt2[CW];
        bool prow = false;
        if constexpr (PML) {
            prow = pstrip || pml_row(A, z);
            if (prow) {
                PmlRow pr;
                pr.init(A, z);
                if (z == W.z0 && z >= 1) {
                    // the edges above the first row, from their previous level
                    PmlRow pu;
                    pu.init(A, z - 1);
#pragma unroll
                    for (int k = 0; k < CW; ++k)
                        pup[k] = pml_edge(pup_old[k], pu.bze, pu.gze, A.hd0 * float(pc.mxc[k] - pu.mze),
                                          q[4][k] - q[3][k], A.ih);
                }
                pml_row_terms<CW>(A, pc, pr, lane, q, xr, c.px, c.pz, c.pxl, pnx, pnz, pup, pdiv);
#pragma unroll
                for (int k = 0; k < CW; ++k) fdt2[k] = (pc.dxc[k] * pr.dzc) * A.dt2;
            } else {
#pragma unroll
                for (int k = 0; k < CW; ++k) pup[k] = 0.f;
            }
        }
        float out[CW], Dv[CW];
#pragma unroll
        for (int k = 0; k < CW; ++k) {
            float lap = lap8(q, xr, k, A.w1, A.w2, A.w3, A.w4);
            if constexpr (PML)
                if (prow) lap = __builtin_fmaf(pdiv[k], A.ih, lap);
            if (FL & F_SRC) lap = add_source<CW>(lap, wsrc, z, S.src_i, sw0, sw1, k);
            if (FL & F_INJECT)
                if (qi[k] >= 0) lap += iv[k];
            const float cc = c.v[k] * c.v[k] * A.dt2;
            float a = ax[k], sh = shx[k];
            if (ddz > 0) {
                sh = A.hs * (dz2 + dx2[k]);
                a = sponge_a(sh);
            }
            Dv[k] = cc * lap;
            // scattered field: the linearised velocity term (2 dV / V) D^n;
            // a relative perturbation dm = dV / V enters as 2 dm D^n
            if (FL & F_SCAT) {
                const float rho = A.rel ? 2.0f * c.dv[k] : 2.0f * c.dv[k] / c.v[k];
                Dv[k] = __builtin_fmaf(rho, c.d[k], Dv[k]);
            }
            float Du = Dv[k];
            if constexpr (PML)
                if (prow) Du = __builtin_fmaf(-fdt2[k], q[4][k], Du);
            out[k] = leapfrog(q[4][k], c.pv[k], Du, a, sh);
            if (A.fs && z == 0) out[k] = 0.0f;   // the pressure-free surface
        }
        const int ro = 4 * (z + kRowsAbove) * P, go = 4 * z * P;
        if (FL & F_EMIT) bst_stream<CW>(rd, js, go, Dv, valid);
        if constexpr (PML) {
            if (prow) {
#pragma unroll
                for (int k = 0; k < CW; ++k) {
                    bst1(rpxo, jsv[k], ro, pnx[k]);
                    bst1(rpzo, jsv[k], ro, pnz[k]);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < CW; ++k) {
            bst1(rprev, jsv[k], ro, out[k]);
            if (FL & F_IMAGE) bst1(rg, jsv[k], go, __builtin_fmaf(out[k], c.d[k], c.g[k]));
            if (FL & F_SAMPLE)
                if (valid[k] && qi[k] >= 0) A.samp[qi[k]] = out[k];
            // odd mirror above the free surface: rows -1..-4 of the new level
            if (A.fs && z >= 1 && z <= kHalo) bst1(rprev, jsv[k], 4 * (kRowsAbove - z) * P, -out[k]);
        }
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int k = 0; k < CW; ++k) q[r][k] = q[r + 1][k];
    };

    // a ring of PD+1 buffers, statically indexed: the loop is unrolled PD+1
    // times so that no buffer is copied. Every pass of the main loop issues
    // the same loads (rows past the run's last are fetched as that row again:
    // cache hits, never used), so the compiler counts the loads in flight
    // exactly and waits for the current row's only; the last rows (fewer than
    // PD+1) are in the ring already.
    Pre buf[PD + 1];
    const int zl = W.z1 - 1;
#pragma unroll
    for (int u = 0; u < PD; ++u) prefetch(min(W.z0 + u, zl), buf[u]);
    int z = W.z0;
    for (; z + PD < W.z1; z += PD + 1) {
#pragma unroll
        for (int u = 0; u <= PD; ++u) {
            prefetch(min(z + u + PD, zl), buf[(u + PD) % (PD + 1)]);
            do_row(z + u, buf[u]);
        }
    }
#pragma unroll
    for (int u = 0; u < PD; ++u)
        if (z + u < W.z1) do_row(z + u, buf[u]);
}

// Two time levels per launch (temporal blocking). With u^{n-1} (prev) and
// u^n (cur) it produces u^{n+1} (out1) and u^{n+2} (out2); run backward in
// time with the residual as source it produces lambda^n and lambda^{n-1};
// with F_SCAT it advances the scattered field driven by the stored D^n and
// D^{n+1} of the background.
// The lanes hold the owned columns plus 4 on each side; level 1 is computed
// on all of them (and on 4 extra rows above and below the owned rows), so
// level 2 can be computed on the owned cells without exchanging data with
// other waves. Level 2 lags level 1 by 4 rows in the z stream. Level 1
// outside the padded box is zero (the Dirichlet halo), as in the one-level
// kernel. Per owned cell and two updates the kernel moves u^n, u^{n-1}, v
// in and u^{n+1}, u^{n+2} out (plus D and G traffic for the adjoint), where
// two one-level launches would move twice as much. The loads of the next PD
// rows are in flight while a row is computed (a ring of PD + 1 statically
// indexed register buffers, as in k_step). Under a free surface (FS) both levels
// are pinned to zero on row 0, and the odd mirror above it is formed inside
// the launch for level 1: when level-1 row m (1..4) is computed, its negative
// goes into the window slot of row -m, which level 2 reads only later; both
// new levels are also stored with their mirrored rows, as k_step stores them.
// With the perfectly matched layer (PML) the edge fields of level n are read
// and those of level n+2 written; the intermediate level's edge fields are
// formed by level 1 on every lane column and row it computes (edges outside
// the box are zero) and reach level 2, four rows later, through register
// rings (the z edges keep one row more: the first level-2 row of a wave also
// needs the edge above it). Level 2's edge left of lane 0 would need level
// 1's edge one column further left; that lane's column is never owned, so
// it is formed from zero.
template <int FL, int CW, int PD, bool FS, bool PML>
__global__ __launch_bounds__(kLanes *kWavesPerBlock) void k_step2(const StepArgs A)
{
    constexpr int SW = kLanes * CW;           // lane columns
    constexpr int RW = SW + 2 * kHalo;
    __shared__ float lds[kWavesPerBlock][2][RW];
    const int lane = threadIdx.x & (kLanes - 1);
    const int wl = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);   // wave-uniform
    const int wid = xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wl;
    if (wid >= A.nwaves) return;
    float *row0 = lds[wl][0];                 // level n, row t (+ 4-column halos)
    float *row1 = lds[wl][1];                 // level 1, row t-4
    const WaveDesc W = A.waves[wid];
    const ShotDesc S = A.shots[W.shot];
    const int P = S.P, nb = A.nb, NZ = A.NZ;
    const int cb = W.col0 - kHalo;            // column of lane 0
    const int j0 = cb + CW * lane;
    // loads are unconditional: negative columns read the previous row's zero
    // tail, columns past the shot's width a zero column
    const int jl = j0 < 0 ? j0 : min(j0, P - 2);
    // byte offsets of the buffer accesses: columns shifted up by 4 (loads of
    // negative columns, row offsets lowered by as much) so that they are
    // never negative
    const unsigned jl4 = 4u * unsigned(jl + kHalo);
    const unsigned js4 = 4u * unsigned(max(j0, 0));    // stores: owned columns only
    const int own_hi = min(W.col0 + SW - 2 * kHalo, S.NX);
    const bool lvl1_ok = A.n < S.nt, lvl2_ok = A.n2 < S.nt;
    const int64_t base = S.f_off - int64_t(kRowsAbove) * P;
    const Rsrc run = view(A.cur + base), rum = view(A.prev + base), rv = view(A.v);
    const Rsrc ro1 = view(A.out1 + base), ro2 = view(A.out2 + base);
    const Rsrc rg = view((FL & F_IMAGE) ? A.G + S.g_off : A.v);
    const Rsrc rd1 = view((FL & (F_IMAGE | F_EMIT | F_SCAT)) ? A.dslot + S.g_off : A.v);
    const Rsrc rd2 = view((FL & (F_IMAGE | F_EMIT | F_SCAT)) ? A.dslot2 + S.g_off : A.v);
    const Rsrc rdv = view((FL & F_SCAT) ? A.dv : A.v);

    bool inbox[CW], own[CW];
    unsigned jso[CW];
    unsigned jm[CW];
    float dx2[CW], ax[CW], shx[CW];
#pragma unroll
    for (int k = 0; k < CW; ++k) {
        const int j = j0 + k;
        inbox[k] = j >= 0 && j < S.NX;
        own[k] = j >= W.col0 && j < own_hi;
        // store offset of the column: past the range (stores dropped) unless owned
        jso[k] = own[k] ? 4u * unsigned(j) : kNoLoad;
        jm[k] = 4u * unsigned(S.x0 + clampi(j - nb, 0, S.wnx - 1));
        const int ddx = max(max(nb - j, j - (S.NX - 1 - nb)), 0);
        dx2[k] = float(ddx * ddx);
        const float sh = A.hs * dx2[k];
        ax[k] = sponge_a(sh);
        shx[k] = sh;
    }
    // halo columns (byte offset shifted up by 8 columns: cb - 4 >= -8)
    const unsigned hcol4 =
        lane < 2 ? 4u * unsigned((lane == 0 ? cb - kHalo : min(cb + SW, P - kHalo)) + 2 * kHalo) : kNoLoad;
    if (lane < 2) *reinterpret_cast<float4 *>(&row1[lane == 0 ? 0 : kHalo + SW]) = make_float4(0.f, 0.f, 0.f, 0.f);

    const int t0 = W.z0 - kHalo, t1 = W.z1 + kHalo;   // level-1 rows [t0, t1)

    // perfectly matched layer: coefficients of the lane columns, the edge
    // fields of the row above the current one at each level, and the rings
    // carrying level 1's edge fields to level 2 (slot 4 / 5: row t)
    PmlCols<CW> pc;
    bool pstrip = false;
    Rsrc rpxi = rv, rpzi = rv, rpxo = rv, rpzo = rv;
    float pup1[CW], pup1_old[CW], pup2[CW], pxr[5][CW], pzr[6][CW];
    const unsigned jleft4 = 4u * unsigned(max(cb - 1, 0) + kHalo);
    if constexpr (PML) {
        pc.init(A, j0, S.NX);
        pstrip = pml_strip<CW>(A, cb, S.NX);
        rpxi = view(A.psx_in + base);
        rpzi = view(A.psz_in + base);
        rpxo = view(A.psx_out + base);
        rpzo = view(A.psz_out + base);
#pragma unroll
        for (int k = 0; k < CW; ++k) {
            pup1[k] = pup1_old[k] = pup2[k] = 0.f;
#pragma unroll
            for (int r = 0; r < 5; ++r) pxr[r][k] = 0.f;
#pragma unroll
            for (int r = 0; r < 6; ++r) pzr[r][k] = 0.f;
        }
        if ((pstrip || pml_row(A, t0)) && t0 >= 1)
            bld<CW>(rpzi, jl4, 4 * ((t0 - 1 + kRowsAbove) * P - kHalo), pup1_old);
    }

    float qa[9][CW], qb[9][CW], cq[5][CW], crho[5][CW];
#pragma unroll
    for (int r = 0; r < 8; ++r) bld<CW>(run, jl4, 4 * ((t0 - kHalo + r + kRowsAbove) * P - kHalo), qa[r]);
#pragma unroll
    for (int r = 0; r < 9; ++r)
#pragma unroll
        for (int k = 0; k < CW; ++k) qb[r][k] = 0.f;
#pragma unroll
    for (int r = 0; r < 5; ++r)
#pragma unroll
        for (int k = 0; k < CW; ++k) cq[r][k] = crho[r][k] = 0.f;

    // the loads of one level-1 row: u^n four rows below it (and its halo
    // columns), u^{n-1}, the model, and for the adjoint D and G of row t-4
    struct Pre2 {
        float q[CW], pv[CW], v[CW], d1[CW], d2[CW], g[CW], dv[CW];
        float px[CW], pz[CW], pxl;
        float4 h;
    };
    const unsigned jc4 = 4u * unsigned(min(max(jl, 0), P - CW));
    auto prefetch = [&](int t, Pre2 &o) {
        const int ro = 4 * ((t + kRowsAbove) * P - kHalo);
        bld<CW>(run, jl4, ro + 4 * kHalo * P, o.q);
        bld<CW>(rum, jl4, ro, o.pv);
        o.h = bld4(run, hcol4, ro - 4 * kHalo);   // zeros past lane 1
        const int vo = 4 * clampi(t - A.top, 0, A.nz - 1) * A.nx;
#pragma unroll
        for (int k = 0; k < CW; ++k) o.v[k] = bld1(rv, jm[k], vo);
        if (FL & F_IMAGE) {
            // the imaging terms of both levels are added at level 2 (row t-4,
            // always below z1); before the first owned row the loads take a
            // lane offset past the range (zeros, no memory request), so that
            // they sit in no branch
            const unsigned jo = t - kHalo >= W.z0 ? jc4 : kNoLoad;
            const int r2 = max(t - kHalo, W.z0);
            bld_stream<CW>(rd1, jo, 4 * r2 * P, o.d1);
            bld_stream<CW>(rd2, jo, 4 * r2 * P, o.d2);
            bld<CW>(rg, jo, 4 * r2 * P, o.g);
        }
        if (FL & F_SCAT) {
            // the scattered field's source: D^n of row t on the lane columns
            // for level 1 (zeros on rows outside the box, where level 1 is
            // zero), D^{n+1} of row t-4 for level 2 (owned rows), dV of row t
            bld_stream<CW>(rd1, t >= 0 && t < NZ ? jc4 : kNoLoad, 4 * clampi(t, 0, NZ - 1) * P, o.d1);
            bld_stream<CW>(rd2, t - kHalo >= W.z0 ? jc4 : kNoLoad, 4 * max(t - kHalo, W.z0) * P, o.d2);
#pragma unroll
            for (int k = 0; k < CW; ++k) o.dv[k] = bld1(rdv, jm[k], vo);
        }
        if constexpr (PML) {
            if (pstrip || pml_row(A, t)) {
                bld<CW>(rpxi, jl4, ro, o.px);
                bld<CW>(rpzi, jl4, ro, o.pz);
                o.pxl = lane == 0 ? bld1(rpxi, jleft4, ro) : 0.f;
            }
        }
    };

    const RecRowsK rrows = rec_rows(A.rrows);
    int rr1 = W.rr0, rr2 = W.rr0;
    int rrow1 = kNoRow, rrow2 = kNoRow;
    if (FL & (F_SAMPLE | F_INJECT)) {
        // skip receiver rows above the first level-1 row
        while (rr1 < W.rr1 && rrows[rr1].row < t0) ++rr1;
        rrow1 = rr1 < W.rr1 ? rrows[rr1].row : kNoRow;
        rr2 = rr1;
        rrow2 = rrow1;
    }
    const float wsrc1 = (FL & F_SRC) ? A.wav[S.wav_off + A.n] * A.ih2 : 0.0f;
    const float wsrc2 = (FL & F_SRC) && lvl2_ok ? A.wav[S.wav_off + A.n2] * A.ih2 : 0.0f;
    const int src_k = S.src_j - j0;
    float sw0[CW], sw1[CW];
    if (FL & F_SRC) source_weights<CW>(S, src_k, sw0, sw1);

    auto do_row = [&](int t, const Pre2 &pf) {
        float cpv[CW], cv[CW], cd1[CW], cd2[CW], cg[CW];
#pragma unroll
        for (int k = 0; k < CW; ++k) {
            qa[8][k] = pf.q[k];
            cpv[k] = pf.pv[k];
            cv[k] = pf.v[k];
            if (FL & F_IMAGE) {
                cd1[k] = pf.d1[k];
                cd2[k] = pf.d2[k];
                cg[k] = pf.g[k];
            }
        }
        const float4 ch = pf.h;

        // ---- level 1 at row t ----------------------------------------------
        if constexpr (CW == 1) row0[kHalo + lane] = qa[4][0];
        else *reinterpret_cast<float2 *>(&row0[kHalo + CW * lane]) = make_float2(qa[4][0], qa[4][1]);
        if (lane < 2) *reinterpret_cast<float4 *>(&row0[lane == 0 ? 0 : kHalo + SW]) = ch;
        wave_sync();
        float xr[CW + 2 * kHalo];
#pragma unroll
        for (int m = 0; m < CW + 2 * kHalo; ++m) xr[m] = row0[CW * lane + m];

        int qi1[CW];
        float iv1[CW];
#pragma unroll
        for (int k = 0; k < CW; ++k) {
            qi1[k] = -1;
            iv1[k] = 0.f;
        }
        if (FL & (F_SAMPLE | F_INJECT))
            if (t == rrow1)
                receiver_row<CW, (FL & F_INJECT) != 0>(A, rrows, A.inj, rr1, rrow1, W.rr1, lane, qi1, iv1);
        const bool row_in = t >= 0 && t < NZ;
        const int ddz1 = max(max(A.top - t, t - (NZ - 1 - nb)), 0);
        const float dz1 = float(ddz1 * ddz1);
        // layer terms of level 1 (as k_step forms them); edges of rows
        // outside the box are zero
        float pdiv1[CW], pnx1[CW], pnz1[CW], fdt1[CW];
        bool prow1 = false;
        if constexpr (PML) {
            prow1 = pstrip || pml_row(A, t);
            if (prow1) {
                PmlRow pr;
                pr.init(A, t);
                if (t == t0 && t >= 1) {
                    PmlRow pu;
                    pu.init(A, t - 1);
#pragma unroll
                    for (int k = 0; k < CW; ++k)
                        pup1[k] = pml_edge(pup1_old[k], pu.bze, pu.gze, A.hd0 * float(pc.mxc[k] - pu.mze),
                                           qa[4][k] - qa[3][k], A.ih);
                }
                pml_row_terms<CW>(A, pc, pr, lane, qa, xr, pf.px, pf.pz, pf.pxl, pnx1, pnz1, pup1, pdiv1);
#pragma unroll
                for (int k = 0; k < CW; ++k) {
                    fdt1[k] = (pc.dxc[k] * pr.dzc) * A.dt2;
                    if (!row_in) pnx1[k] = pnz1[k] = pup1[k] = 0.f;
                }
            } else {
#pragma unroll
                for (int k = 0; k < CW; ++k) pnx1[k] = pnz1[k] = pup1[k] = 0.f;
            }
#pragma unroll
            for (int k = 0; k < CW; ++k) {
                pxr[4][k] = pnx1[k];
                pzr[5][k] = pnz1[k];
            }
        }
        float v1[CW], D1[CW];
#pragma unroll
        for (int k = 0; k < CW; ++k) {
            float lap = lap8(qa, xr, k, A.w1, A.w2, A.w3, A.w4);
            if constexpr (PML)
                if (prow1) lap = __builtin_fmaf(pdiv1[k], A.ih, lap);
            if (FL & F_SRC) lap = add_source<CW>(lap, wsrc1, t, S.src_i, sw0, sw1, k);
            if (FL & F_INJECT)
                if (qi1[k] >= 0) lap += iv1[k];
            const float c = cv[k] * cv[k] * A.dt2;
            float a = ax[k], sh = shx[k];
            if (ddz1 > 0) {
                sh = A.hs * (dz1 + dx2[k]);
                a = sponge_a(sh);
            }
            D1[k] = c * lap;
            // scattered field: the linearised velocity term, as in k_step;
            // the factor travels to level 2 with the row
            if (FL & F_SCAT) {
                const float rho = A.rel ? 2.0f * pf.dv[k] : 2.0f * pf.dv[k] / cv[k];
                crho[4][k] = rho;
                D1[k] = __builtin_fmaf(rho, pf.d1[k], D1[k]);
            }
            float Du = D1[k];
            if constexpr (PML)
                if (prow1) Du = __builtin_fmaf(-fdt1[k], qa[4][k], Du);
            const float o = leapfrog(qa[4][k], cpv[k], Du, a, sh);
            v1[k] = (row_in && inbox[k]) ? o : 0.0f;
            if (FS && t == 0) v1[k] = 0.0f;   // the pressure-free surface
            qb[8][k] = v1[k];
            cq[4][k] = c;
        }
        if (FS && t >= 1 && t <= kHalo) {
            // level 1 above the surface: the odd mirror of rows 1..4, in the
            // slot of row -t (the window holds rows t-8 .. t)
#pragma unroll
            for (int k = 0; k < CW; ++k) {
                const float m = -v1[k];
                if (t == 1) qb[6][k] = m;
                else if (t == 2) qb[4][k] = m;
                else if (t == 3) qb[2][k] = m;
                else qb[0][k] = m;
            }
        }
        const bool own_row1 = t >= W.z0 && t < W.z1;
        if (own_row1) {
            const int o = 4 * (t + kRowsAbove) * P;
            if (FL & F_EMIT) bst_stream<CW>(rd1, js4, 4 * t * P, D1, own);
#pragma unroll
            for (int k = 0; k < CW; ++k) {
                bst1(ro1, jso[k], o, v1[k]);
                if (FS && t >= 1 && t <= kHalo) bst1(ro1, jso[k], 4 * (kRowsAbove - t) * P, -v1[k]);
                if (FL & F_SAMPLE)
                    if (own[k] && qi1[k] >= 0) A.samp[qi1[k]] = v1[k];
            }
        }

        // ---- level 2 at row t-4 -------------------------------------------
        const int r2 = t - kHalo;
        if constexpr (CW == 1) row1[kHalo + lane] = qb[4][0];
        else *reinterpret_cast<float2 *>(&row1[kHalo + CW * lane]) = make_float2(qb[4][0], qb[4][1]);
        wave_sync();
        float yr[CW + 2 * kHalo];
#pragma unroll
        for (int m = 0; m < CW + 2 * kHalo; ++m) yr[m] = row1[CW * lane + m];
        wave_sync();

        int qi2[CW];
        float iv2[CW];
#pragma unroll
        for (int k = 0; k < CW; ++k) {
            qi2[k] = -1;
            iv2[k] = 0.f;
        }
        if (FL & (F_SAMPLE | F_INJECT))
            if (r2 == rrow2)
                receiver_row<CW, (FL & F_INJECT) != 0>(A, rrows, A.inj2, rr2, rrow2, W.rr1, lane, qi2, iv2);
        if (r2 >= W.z0) {   // r2 < z1 always holds
            const int ddz2 = max(max(A.top - r2, r2 - (NZ - 1 - nb)), 0);
            const float dz2 = float(ddz2 * ddz2);
            const int o = 4 * (r2 + kRowsAbove) * P;
            // layer terms of level 2 from level 1's edge fields of row r2
            // (and, for the first row, of the row above it)
            float pdiv2[CW], pnx2[CW], pnz2[CW], fdt2[CW];
            bool prow2 = false;
            if constexpr (PML) {
                prow2 = pstrip || pml_row(A, r2);
                if (prow2) {
                    PmlRow pr;
                    pr.init(A, r2);
                    if (r2 == W.z0 && r2 >= 1) {
                        PmlRow pu;
                        pu.init(A, r2 - 1);
#pragma unroll
                        for (int k = 0; k < CW; ++k)
                            pup2[k] = pml_edge(pzr[0][k], pu.bze, pu.gze, A.hd0 * float(pc.mxc[k] - pu.mze),
                                               qb[4][k] - qb[3][k], A.ih);
                    }
                    pml_row_terms<CW>(A, pc, pr, lane, qb, yr, pxr[0], pzr[1], 0.f, pnx2, pnz2, pup2, pdiv2);
#pragma unroll
                    for (int k = 0; k < CW; ++k) fdt2[k] = (pc.dxc[k] * pr.dzc) * A.dt2;
                } else {
#pragma unroll
                    for (int k = 0; k < CW; ++k) pup2[k] = 0.f;
                }
            }
            float D2[CW];
#pragma unroll
            for (int k = 0; k < CW; ++k) {
                float lap = lap8(qb, yr, k, A.w1, A.w2, A.w3, A.w4);
                if constexpr (PML)
                    if (prow2) lap = __builtin_fmaf(pdiv2[k], A.ih, lap);
                if (FL & F_SRC) lap = add_source<CW>(lap, wsrc2, r2, S.src_i, sw0, sw1, k);
                if (FL & F_INJECT)
                    if (qi2[k] >= 0) lap += iv2[k];
                const float c = cq[0][k];
                float a = ax[k], sh = shx[k];
                if (ddz2 > 0) {
                    sh = A.hs * (dz2 + dx2[k]);
                    a = sponge_a(sh);
                }
                D2[k] = c * lap;
                if (FL & F_SCAT) D2[k] = __builtin_fmaf(crho[0][k], pf.d2[k], D2[k]);
                float Du = D2[k];
                if constexpr (PML)
                    if (prow2) Du = __builtin_fmaf(-fdt2[k], qb[4][k], Du);
                float v2 = leapfrog(qb[4][k], qa[0][k], Du, a, sh);
                if (FS && r2 == 0) v2 = 0.0f;   // the pressure-free surface
                bst1(ro2, jso[k], o, v2);
                if constexpr (PML) {
                    if (prow2) {
                        bst1(rpxo, jso[k], o, pnx2[k]);
                        bst1(rpzo, jso[k], o, pnz2[k]);
                    }
                }
                if (FS && r2 >= 1 && r2 <= kHalo) bst1(ro2, jso[k], 4 * (kRowsAbove - r2) * P, -v2);
                if (FL & F_SAMPLE)
                    if (own[k] && lvl2_ok && qi2[k] >= 0) A.samp2[qi2[k]] = v2;
                // G after both levels: the fused multiply-adds of two one-level
                // steps, in their order (qb[4] is the level-1 value of this row)
                if (FL & F_IMAGE) {
                    const float g1 = lvl1_ok ? __builtin_fmaf(qb[4][k], cd1[k], cg[k]) : cg[k];
                    bst1(rg, jso[k], 4 * r2 * P, __builtin_fmaf(v2, cd2[k], g1));
                }
            }
            if (FL & F_EMIT)
                if (lvl2_ok) bst_stream<CW>(rd2, js4, 4 * r2 * P, D2, own);
        }
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int k = 0; k < CW; ++k) {
                qa[r][k] = qa[r + 1][k];
                qb[r][k] = qb[r + 1][k];
            }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int k = 0; k < CW; ++k) {
                cq[r][k] = cq[r + 1][k];
                if (FL & F_SCAT) crho[r][k] = crho[r + 1][k];
            }
        if constexpr (PML) {
#pragma unroll
            for (int k = 0; k < CW; ++k) {
#pragma unroll
                for (int r = 0; r < 4; ++r) pxr[r][k] = pxr[r + 1][k];
#pragma unroll
                for (int r = 0; r < 5; ++r) pzr[r][k] = pzr[r + 1][k];
            }
        }
    };

    // the ring and loop structure of k_step
    Pre2 buf[PD + 1];
    const int tl = t1 - 1;
#pragma unroll
    for (int u = 0; u < PD; ++u) prefetch(min(t0 + u, tl), buf[u]);
    int t = t0;
    for (; t + PD < t1; t += PD + 1) {
#pragma unroll
        for (int u = 0; u <= PD; ++u) {
            prefetch(min(t + u + PD, tl), buf[(u + PD) % (PD + 1)]);
            do_row(t + u, buf[u]);
        }
    }
#pragma unroll
    for (int u = 0; u < PD; ++u)
        if (t + u < t1) do_row(t + u, buf[u]);
}

// Born: background u and scattered du advanced together (section 2.2: the
// two equations are solved jointly so that u is never stored):
//   du^{n+1} = a (2 du^n + V^2 dt^2 L8 du^n + 2 V dV dt^2 (L8 u^n + s^n)) - b du^{n-1}
// where 2 V dV dt^2 = (2 dV / V) V^2 dt^2 is the linearised 1/V^2 term.
// Same tiling and prefetching as k_step; receivers record du^{n+1}. With
// EMIT the background's D^n = V^2 dt^2 (L8 u^n + s^n) is also written to the
// D slot (the same value the forward step emits), so that a migration can
// follow without a separate background sweep.
template <int CW, bool EMIT, bool PML>
__global__ __launch_bounds__(kLanes *kWavesPerBlock) void k_born_step(const StepArgs A)
{
    constexpr int SW = kLanes * CW;
    constexpr int RW = SW + 2 * kHalo;
    __shared__ float lds[kWavesPerBlock][2][RW];
    const int lane = threadIdx.x & (kLanes - 1);
    const int wl = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);   // wave-uniform
    const int wid = xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wl;
    if (wid >= A.nwaves) return;
    float *row = lds[wl][0];
    float *rod = lds[wl][1];
    const WaveDesc W = A.waves[wid];
    const ShotDesc S = A.shots[W.shot];
    const int P = S.P;
    const int nb = A.nb;
    const int j0 = W.col0 + CW * lane;
    const unsigned jl = 4u * unsigned(min(j0, P - 2));   // byte offsets
    const unsigned js = 4u * unsigned(j0);
    const int64_t base = S.f_off - int64_t(kRowsAbove) * P;
    const Rsrc rcu = view(A.cur + base), rpv = view(A.prev + base);
    const Rsrc rcd = view(A.cur2 + base), rpd = view(A.prev2 + base);
    const Rsrc rv = view(A.v), rdv = view(A.dv);
    const Rsrc rd = view(EMIT ? A.dslot + S.g_off : A.v);

    bool valid[CW];
    unsigned jm[CW];
    float dx2[CW], ax[CW], shx[CW];
#pragma unroll
    for (int k = 0; k < CW; ++k) {
        const int j = j0 + k;
        valid[k] = j < S.NX;
        jm[k] = 4u * unsigned(S.x0 + clampi(j - nb, 0, S.wnx - 1));
        const int ddx = max(max(nb - j, j - (S.NX - 1 - nb)), 0);
        dx2[k] = float(ddx * ddx);
        const float sh = A.hs * dx2[k];
        ax[k] = sponge_a(sh);
        shx[k] = sh;
    }
    // halo columns (byte offset shifted up by 4 columns, row offset lowered)
    const unsigned hcol =
        lane < 2 ? 4u * unsigned(lane == 0 ? W.col0 : min(W.col0 + SW, P - kHalo) + kHalo) : kNoLoad;

    // perfectly matched layer: edge fields of u (psx, psz) and du (psx2, psz2)
    PmlCols<CW> pc;
    bool pstrip = false;
    Rsrc rpxi = rv, rpzi = rv, rpxo = rv, rpzo = rv, rqxi = rv, rqzi = rv, rqxo = rv, rqzo = rv;
    float pup[CW], pup_old[CW], qup[CW], qup_old[CW];
    const unsigned jleft = 4u * unsigned(max(W.col0 - 1, 0));
    if constexpr (PML) {
        pc.init(A, j0, S.NX);
        pstrip = pml_strip<CW>(A, W.col0, S.NX);
        rpxi = view(A.psx_in + base);
        rpzi = view(A.psz_in + base);
        rpxo = view(A.psx_out + base);
        rpzo = view(A.psz_out + base);
        rqxi = view(A.psx2_in + base);
        rqzi = view(A.psz2_in + base);
        rqxo = view(A.psx2_out + base);
        rqzo = view(A.psz2_out + base);
#pragma unroll
        for (int k = 0; k < CW; ++k) pup[k] = pup_old[k] = qup[k] = qup_old[k] = 0.f;
        if ((pstrip || pml_row(A, W.z0)) && W.z0 >= 1) {
            bld<CW>(rpzi, jl, 4 * (W.z0 - 1 + kRowsAbove) * P, pup_old);
            bld<CW>(rqzi, jl, 4 * (W.z0 - 1 + kRowsAbove) * P, qup_old);
        }
    }

    float q[9][CW], r[9][CW];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        bld<CW>(rcu, jl, 4 * (W.z0 - kHalo + k + kRowsAbove) * P, q[k]);
        bld<CW>(rcd, jl, 4 * (W.z0 - kHalo + k + kRowsAbove) * P, r[k]);
    }
    float nq[CW], nr[CW], npv[CW], npd[CW], nv[CW], ndv[CW];
    float npx[CW], npz[CW], nqx[CW], nqz[CW], npxl = 0.f, nqxl = 0.f;
    float4 nh = make_float4(0.f, 0.f, 0.f, 0.f), nhd = nh;
    auto prefetch = [&](int z) {
        const int ro = 4 * (z + kRowsAbove) * P;
        bld<CW>(rcu, jl, ro + 4 * kHalo * P, nq);
        bld<CW>(rcd, jl, ro + 4 * kHalo * P, nr);
        bld<CW>(rpv, jl, ro, npv);
        bld<CW>(rpd, jl, ro, npd);
        nh = bld4(rcu, hcol, ro - 4 * kHalo);     // zeros past lane 1
        nhd = bld4(rcd, hcol, ro - 4 * kHalo);
        const int vo = 4 * clampi(z - A.top, 0, A.nz - 1) * A.nx;
#pragma unroll
        for (int k = 0; k < CW; ++k) {
            nv[k] = bld1(rv, jm[k], vo);
            ndv[k] = bld1(rdv, jm[k], vo);
        }
        if constexpr (PML) {
            if (pstrip || pml_row(A, z)) {
                bld<CW>(rpxi, jl, ro, npx);
                bld<CW>(rpzi, jl, ro, npz);
                bld<CW>(rqxi, jl, ro, nqx);
                bld<CW>(rqzi, jl, ro, nqz);
                npxl = lane == 0 ? bld1(rpxi, jleft, ro) : 0.f;
                nqxl = lane == 0 ? bld1(rqxi, jleft, ro) : 0.f;
            }
        }
    };
    prefetch(W.z0);

    const RecRowsK rrows = rec_rows(A.rrows);
    int rr = W.rr0;
    int rrow = rr < W.rr1 ? rrows[rr].row : kNoRow;
    const float wsrc = A.wav[S.wav_off + A.n] * A.ih2;
    const int src_k = S.src_j - j0;
    float sw0[CW], sw1[CW];
    source_weights<CW>(S, src_k, sw0, sw1);

    for (int z = W.z0; z < W.z1; ++z) {
        float cpv[CW], cpd[CW], cv[CW], cdv[CW];
        float cpx[CW], cpz[CW], cqx[CW], cqz[CW];
        const float cpxl = npxl, cqxl = nqxl;
#pragma unroll
        for (int k = 0; k < CW; ++k) {
            q[8][k] = nq[k];
            r[8][k] = nr[k];
            cpv[k] = npv[k];
            cpd[k] = npd[k];
            cv[k] = nv[k];
            cdv[k] = ndv[k];
            cpx[k] = npx[k];
            cpz[k] = npz[k];
            cqx[k] = nqx[k];
            cqz[k] = nqz[k];
        }
        const float4 ch = nh, chd = nhd;
        prefetch(min(z + 1, W.z1 - 1));   // past the last row: that row again (unused)

        if constexpr (CW == 1) {
            row[kHalo + lane] = q[4][0];
            rod[kHalo + lane] = r[4][0];
        } else {
            *reinterpret_cast<float2 *>(&row[kHalo + CW * lane]) = make_float2(q[4][0], q[4][1]);
            *reinterpret_cast<float2 *>(&rod[kHalo + CW * lane]) = make_float2(r[4][0], r[4][1]);
        }
        if (lane < 2) {
            *reinterpret_cast<float4 *>(&row[lane == 0 ? 0 : kHalo + SW]) = ch;
            *reinterpret_cast<float4 *>(&rod[lane == 0 ? 0 : kHalo + SW]) = chd;
        }
        wave_sync();
        float xr[CW + 2 * kHalo], xd[CW + 2 * kHalo];
#pragma unroll
        for (int m = 0; m < CW + 2 * kHalo; ++m) {
            xr[m] = row[CW * lane + m];
            xd[m] = rod[CW * lane + m];
        }
        wave_sync();

        int qi[CW];
        float iv[CW];
#pragma unroll
        for (int k = 0; k < CW; ++k) qi[k] = -1;
        if (z == rrow) receiver_row<CW, false>(A, rrows, nullptr, rr, rrow, W.rr1, lane, qi, iv);
        const int ddz = max(max(A.top - z, z - (A.NZ - 1 - nb)), 0);
        const float dz2 = float(ddz * ddz);
        // layer terms of this row for both fields
        float pdiv[CW], pnx[CW], pnz[CW], qdiv[CW], qnx[CW], qnz[CW], fdt2[CW];
        bool prow = false;
        if constexpr (PML) {
            prow = pstrip || pml_row(A, z);
            if (prow) {
                PmlRow pr;
                pr.init(A, z);
                if (z == W.z0 && z >= 1) {
                    PmlRow pu;
                    pu.init(A, z - 1);
#pragma unroll
                    for (int k = 0; k < CW; ++k) {
                        const float ed = A.hd0 * float(pc.mxc[k] - pu.mze);
                        pup[k] = pml_edge(pup_old[k], pu.bze, pu.gze, ed, q[4][k] - q[3][k], A.ih);
                        qup[k] = pml_edge(qup_old[k], pu.bze, pu.gze, ed, r[4][k] - r[3][k], A.ih);
                    }
                }
                pml_row_terms<CW>(A, pc, pr, lane, q, xr, cpx, cpz, cpxl, pnx, pnz, pup, pdiv);
                pml_row_terms<CW>(A, pc, pr, lane, r, xd, cqx, cqz, cqxl, qnx, qnz, qup, qdiv);
#pragma unroll
                for (int k = 0; k < CW; ++k) fdt2[k] = (pc.dxc[k] * pr.dzc) * A.dt2;
            } else {
#pragma unroll
                for (int k = 0; k < CW; ++k) pup[k] = qup[k] = 0.f;
            }
        }
        float ou[CW], od[CW], Dv[CW];
#pragma unroll
        for (int k = 0; k < CW; ++k) {
            float lap = lap8(q, xr, k, A.w1, A.w2, A.w3, A.w4);
            float lapd = lap8(r, xd, k, A.w1, A.w2, A.w3, A.w4);
            if constexpr (PML) {
                if (prow) {
                    lap = __builtin_fmaf(pdiv[k], A.ih, lap);
                    lapd = __builtin_fmaf(qdiv[k], A.ih, lapd);
                }
            }
            lap = add_source<CW>(lap, wsrc, z, S.src_i, sw0, sw1, k);
            const float c = cv[k] * cv[k] * A.dt2;
            // (2 dV / V) V^2 dt^2, or 2 dm V^2 dt^2 for a relative dm
            const float cr = A.rel ? 2.0f * cdv[k] * c : 2.0f * cv[k] * cdv[k] * A.dt2;
            float a = ax[k], sh = shx[k];
            if (ddz > 0) {
                sh = A.hs * (dz2 + dx2[k]);
                a = sponge_a(sh);
            }
            Dv[k] = c * lap;
            float Du = Dv[k], Dd = __builtin_fmaf(cr, lap, c * lapd);
            if constexpr (PML) {
                if (prow) {
                    Du = __builtin_fmaf(-fdt2[k], q[4][k], Du);
                    Dd = __builtin_fmaf(-fdt2[k], r[4][k], Dd);
                }
            }
            ou[k] = leapfrog(q[4][k], cpv[k], Du, a, sh);
            od[k] = leapfrog(r[4][k], cpd[k], Dd, a, sh);
            if (A.fs && z == 0) ou[k] = od[k] = 0.0f;   // the pressure-free surface
        }
        const int o = 4 * (z + kRowsAbove) * P;
        if (EMIT) bst_stream<CW>(rd, js, 4 * z * P, Dv, valid);
        if constexpr (PML) {
            if (prow) {
#pragma unroll
                for (int k = 0; k < CW; ++k)
                    if (valid[k]) {
                        bst1(rpxo, js + 4 * k, o, pnx[k]);
                        bst1(rpzo, js + 4 * k, o, pnz[k]);
                        bst1(rqxo, js + 4 * k, o, qnx[k]);
                        bst1(rqzo, js + 4 * k, o, qnz[k]);
                    }
            }
        }
#pragma unroll
        for (int k = 0; k < CW; ++k) {
            if (valid[k]) {
                bst1(rpv, js + 4 * k, o, ou[k]);
                bst1(rpd, js + 4 * k, o, od[k]);
                if (qi[k] >= 0) A.samp[qi[k]] = od[k];
                if (A.fs && z >= 1 && z <= kHalo) {   // odd mirror above the free surface
                    bst1(rpv, js + 4 * k, 4 * (kRowsAbove - z) * P, -ou[k]);
                    bst1(rpd, js + 4 * k, 4 * (kRowsAbove - z) * P, -od[k]);
                }
            }
        }
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
            for (int k = 0; k < CW; ++k) {
                q[m][k] = q[m + 1][k];
                r[m][k] = r[m + 1][k];
            }
    }
}

__global__ void k_scale(const float *x, float a, float *y, int64_t n)
{
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = a * x[i];
}

__global__ void k_fill(float *p, int64_t n, float val)
{
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = val;
}

// Direct-arrival mute of packed traces (the RTM image product, section 3.3):
// sample n (time n dt) of trace r is weighted by 0 up to t0[r], by a
// half-cosine ramp over the taper, then by 1. One block per trace at a time.
__global__ __launch_bounds__(256) void k_mute(const int64_t *off, const int32_t *nt, const float *t0, int32_t ntr,
                                              float dt, float itaper, const float *din, float *dout)
{
    for (int r = blockIdx.x; r < ntr; r += gridDim.x) {
        const int64_t o = off[r];
        const int32_t n_r = nt[r];
        const float t0r = t0[r];
        for (int n = threadIdx.x; n < n_r; n += blockDim.x) {
            const float u = fminf(fmaxf((float(n) * dt - t0r) * itaper, 0.f), 1.f);
            dout[o + n] = din[o + n] * (0.5f - 0.5f * cospif(u));
        }
    }
}

// y = -(d2/dz2 + d2/dx2) x in grid units: the 5-point Laplacian with zero
// outside the image, [nz][nx] row-major.
__global__ __launch_bounds__(256) void k_laplace5(const float *x, int32_t nz, int32_t nx, float *y)
{
    const int64_t n = int64_t(nz) * nx;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int z = int(i / nx), xj = int(i - int64_t(z) * nx);
        const float up = z > 0 ? x[i - nx] : 0.f, dn = z + 1 < nz ? x[i + nx] : 0.f;
        const float lf = xj > 0 ? x[i - 1] : 0.f, rt = xj + 1 < nx ? x[i + 1] : 0.f;
        y[i] = 4.f * x[i] - ((up + dn) + (lf + rt));
    }
}

// min, max and count of non-finite or non-positive entries of v.
__global__ __launch_bounds__(256) void k_model_check(const float *v, int64_t n, float *out3)
{
    __shared__ float smin[256], smax[256], sbad[256];
    float mn = 3.4e38f, mx = -3.4e38f, bad = 0.0f;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const float x = v[i];
        if (!(x > 0.0f) || !(x < 3.4e38f)) bad += 1.0f;
        else {
            mn = fminf(mn, x);
            mx = fmaxf(mx, x);
        }
    }
    smin[threadIdx.x] = mn;
    smax[threadIdx.x] = mx;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            smin[threadIdx.x] = fminf(smin[threadIdx.x], smin[threadIdx.x + s]);
            smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + s]);
            sbad[threadIdx.x] += sbad[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out3[0] = smin[0];
        out3[1] = smax[0];
        out3[2] = sbad[0];
    }
}

// 64 unique receiver cells x 64 time samples per workgroup of 4 waves.
__global__ __launch_bounds__(256) void k_traces(const TraceArgs A)
{
    __shared__ float T[64][65];
    __shared__ float U[64][65];
    __shared__ double red[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int q0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
    const int qq = q0 + lane;
    const int qnt = qq < A.Q ? A.q_nt[qq] : 0;
    // load the time-major tile (rows n, lanes q)
    for (int nl = w; nl < 64; nl += 4) {
        const int n = n0 + nl;
        float x = 0.0f;
        if (A.tm_in && n < qnt) x = A.tm_in[int64_t(n) * A.Q + qq];
        T[nl][lane] = x;
    }
    __syncthreads();
    double part = 0.0;
    const int n = n0 + lane;
    for (int ql = w; ql < 64; ql += 4) {
        const int q = q0 + ql;
        float acc = 0.0f;
        if (q < A.Q) {
            const int nt = A.q_nt[q];
            const float tv = T[lane][ql];
            const int k1 = A.q_rptr[q + 1];
            for (int k = A.q_rptr[q]; k < k1; ++k) {
                const int64_t off = A.q_roff[k];
                if (n < nt) {
                    float val = A.alpha * tv;
                    if (A.tr_in) val += A.beta * A.tr_in[off + n];
                    if (A.tr_out) A.tr_out[off + n] = tv;
                    acc += val;
                    part += 0.5 * double(val) * double(val);
                }
            }
        }
        U[lane][ql] = acc;
    }
    __syncthreads();
    if (A.tm_out) {
        for (int nl = w; nl < 64; nl += 4) {
            const int nn = n0 + nl;
            if (nn < A.nt_max && qq < A.Q) A.tm_out[int64_t(nn) * A.Q + qq] = U[nl][lane];
        }
    }
    if (A.partials) {
        for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
        if (lane == 0) red[w] = part;
        __syncthreads();
        if (threadIdx.x == 0)
            A.partials[int64_t(blockIdx.y) * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
    }
}

// Off-grid receivers, first pass (grid: receivers x time blocks): the trace
// of receiver r is the weighted sum of its cells' time-major samples;
// tr_out receives it and resid its residual alpha*trace + beta*tr_in.
__global__ __launch_bounds__(256) void k_traces_rec(const TraceArgs A)
{
    const int r = blockIdx.x;
    const int n = blockIdx.y * blockDim.x + threadIdx.x;
    if (n >= A.r_nt[r]) return;
    const int k1 = A.r_cptr[r + 1];
    float s = 0.0f;
    if (A.tm_in)
        for (int k = A.r_cptr[r]; k < k1; ++k)
            s = __builtin_fmaf(A.r_cw[k], A.tm_in[int64_t(n) * A.Q + A.r_cq[k]], s);
    const int64_t off = A.r_off[r];
    if (A.tr_out) A.tr_out[off + n] = s;
    if (A.resid) {
        float val = A.alpha * s;
        if (A.tr_in) val += A.beta * A.tr_in[off + n];
        A.resid[off + n] = val;
    }
}

// Off-grid receivers, second pass (one thread per time-major sample n*Q+q):
// the adjoint source of cell q is the weighted sum of the residuals of the
// receivers that use it (zero past the cell's record length).
__global__ __launch_bounds__(256) void k_traces_cell(const TraceArgs A)
{
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= int64_t(A.nt_max) * A.Q) return;
    const int q = int(e % A.Q), n = int(e / A.Q);
    float acc = 0.0f;
    if (n < A.q_nt[q]) {
        const int k1 = A.q_rptr[q + 1];
        for (int k = A.q_rptr[q]; k < k1; ++k) acc = __builtin_fmaf(A.q_rw[k], A.resid[A.q_roff[k] + n], acc);
    }
    A.tm_out[e] = acc;
}

// partials[block] = 1/2 sum of x^2 over a block-strided share of x (fixed order)
__global__ __launch_bounds__(256) void k_half_sumsq(const float *x, int64_t n, double *partials)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        acc += 0.5 * double(x[i]) * double(x[i]);
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// Deterministic sum of the per-block partials (fixed order).
__global__ __launch_bounds__(256) void k_sum_partials(const double *p, int64_t n, double *out)
{
    __shared__ double s[256];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) acc += p[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

// Pad^T, first half: fold the top and bottom sponge rows of every shot's G
// onto the first and last physical rows (one thread per shot column), then
// the left and right sponge columns onto the first and last physical columns
// (one thread per shot row). In place; a fixed summation order per cell.
__global__ __launch_bounds__(256) void k_fold_rows(const FinalArgs A, int maxNX)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    const ShotDesc S = A.shots[s];
    if (j >= S.NX || A.nb == 0) return;
    float *G = A.G + S.g_off;
    const int top = A.top, bot = A.NZ - 1 - A.nb;
    float t = 0.f, b = 0.f;
    for (int r = 0; r <= A.top; ++r) t += G[int64_t(r) * S.P + j];
    for (int r = 0; r <= A.nb; ++r) b += G[int64_t(bot + r) * S.P + j];
    if (top == bot) {  // one physical row: everything folds onto it
        G[int64_t(top) * S.P + j] = t + b - G[int64_t(top) * S.P + j];
    } else {
        G[int64_t(top) * S.P + j] = t;
        G[int64_t(bot) * S.P + j] = b;
    }
}

__global__ __launch_bounds__(256) void k_fold_cols(const FinalArgs A)
{
    const int i = A.top + blockIdx.x * blockDim.x + threadIdx.x;  // physical rows only
    const int s = blockIdx.y;
    if (i > A.NZ - 1 - A.nb || A.nb == 0) return;
    const ShotDesc S = A.shots[s];
    float *G = A.G + S.g_off + int64_t(i) * S.P;
    const int lft = A.nb, rgt = S.NX - 1 - A.nb;
    float l = 0.f, r = 0.f;
    for (int c = 0; c <= A.nb; ++c) {
        l += G[c];
        r += G[rgt + c];
    }
    if (lft == rgt) {
        G[lft] = l + r - G[lft];
    } else {
        G[lft] = l;
        G[rgt] = r;
    }
}

// img = (2 / (v^3 dt^2)) sum_shots Pad^T G_s, after the sponge folds: each
// physical cell reads one value per shot whose window holds it; shots are
// summed in slot order, so the result does not depend on scheduling.
__global__ __launch_bounds__(256) void k_finalize(const FinalArgs A)
{
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= int64_t(A.nz) * A.nx) return;
    const int i = int(p / A.nx), j = int(p % A.nx);
    float acc = 0.0f;
    for (int s = 0; s < A.nshots; ++s) {
        const ShotDesc S = A.shots[s];
        const int jl = j - S.x0;
        if (jl < 0 || jl >= S.wnx) continue;
        acc += A.G[S.g_off + int64_t(i + A.top) * S.P + jl + A.nb];
    }
    // image of dV: (2 / (V^3 dt^2)) sum G; of the relative dV / V: V times that
    const float v = A.v[p];
    A.img[p] = acc * (A.rel ? 2.0f / (v * v * A.dt2) : 2.0f / (v * v * v * A.dt2));
}

inline int blocks_for(int nwaves) { return (nwaves + kWavesPerBlock - 1) / kWavesPerBlock; }

}  // namespace

template <int CW, int PD, bool PML>
hipError_t launch_step_cw(int flags, const StepArgs &a, hipStream_t s)
{
    const dim3 grid(blocks_for(a.nwaves)), block(kLanes * kWavesPerBlock);
    switch (flags) {
    case F_SRC | F_SAMPLE:
        hipLaunchKernelGGL((k_step<F_SRC | F_SAMPLE, CW, PD, PML>), grid, block, 0, s, a);
        break;
    case F_SRC:
        hipLaunchKernelGGL((k_step<F_SRC, CW, PD, PML>), grid, block, 0, s, a);
        break;
    case F_SRC | F_SAMPLE | F_EMIT:
        hipLaunchKernelGGL((k_step<F_SRC | F_SAMPLE | F_EMIT, CW, PD, PML>), grid, block, 0, s, a);
        break;
    case F_SRC | F_EMIT:
        hipLaunchKernelGGL((k_step<F_SRC | F_EMIT, CW, PD, PML>), grid, block, 0, s, a);
        break;
    case F_INJECT | F_IMAGE:
        hipLaunchKernelGGL((k_step<F_INJECT | F_IMAGE, CW, PD, PML>), grid, block, 0, s, a);
        break;
    case F_SAMPLE | F_SCAT:
        hipLaunchKernelGGL((k_step<F_SAMPLE | F_SCAT, CW, PD, PML>), grid, block, 0, s, a);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <bool PML>
hipError_t launch_step_pml(int flags, const StepArgs &a, hipStream_t s)
{
    if (a.pd == 2)
        return a.cw == 2 ? launch_step_cw<2, 2, PML>(flags, a, s) : launch_step_cw<1, 2, PML>(flags, a, s);
    return a.cw == 2 ? launch_step_cw<2, 1, PML>(flags, a, s) : launch_step_cw<1, 1, PML>(flags, a, s);
}

hipError_t launch_step(int flags, const StepArgs &a, hipStream_t s)
{
    if (a.nwaves <= 0) return hipSuccess;
    return a.pml ? launch_step_pml<true>(flags, a, s) : launch_step_pml<false>(flags, a, s);
}

template <int CW, int PD, bool FS, bool PML>
hipError_t launch_step2_cw(int flags, const StepArgs &a, hipStream_t s)
{
    const dim3 grid(blocks_for(a.nwaves)), block(kLanes * kWavesPerBlock);
    switch (flags) {
    case F_SRC | F_SAMPLE:
        hipLaunchKernelGGL((k_step2<F_SRC | F_SAMPLE, CW, PD, FS, PML>), grid, block, 0, s, a);
        break;
    case F_SRC:
        hipLaunchKernelGGL((k_step2<F_SRC, CW, PD, FS, PML>), grid, block, 0, s, a);
        break;
    case F_SRC | F_SAMPLE | F_EMIT:
        hipLaunchKernelGGL((k_step2<F_SRC | F_SAMPLE | F_EMIT, CW, PD, FS, PML>), grid, block, 0, s, a);
        break;
    case F_SRC | F_EMIT:
        hipLaunchKernelGGL((k_step2<F_SRC | F_EMIT, CW, PD, FS, PML>), grid, block, 0, s, a);
        break;
    case F_INJECT | F_IMAGE:
        hipLaunchKernelGGL((k_step2<F_INJECT | F_IMAGE, CW, PD, FS, PML>), grid, block, 0, s, a);
        break;
    case F_SAMPLE | F_SCAT:
        hipLaunchKernelGGL((k_step2<F_SAMPLE | F_SCAT, CW, PD, FS, PML>), grid, block, 0, s, a);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <bool FS, bool PML>
hipError_t launch_step2_bnd(int flags, const StepArgs &a, hipStream_t s)
{
    if (a.pd == 2)
        return a.cw == 2 ? launch_step2_cw<2, 2, FS, PML>(flags, a, s) : launch_step2_cw<1, 2, FS, PML>(flags, a, s);
    return a.cw == 2 ? launch_step2_cw<2, 1, FS, PML>(flags, a, s) : launch_step2_cw<1, 1, FS, PML>(flags, a, s);
}

hipError_t launch_step2(int flags, const StepArgs &a, hipStream_t s)
{
    if (a.nwaves <= 0) return hipSuccess;
    if (a.pml) return a.fs ? launch_step2_bnd<true, true>(flags, a, s) : launch_step2_bnd<false, true>(flags, a, s);
    return a.fs ? launch_step2_bnd<true, false>(flags, a, s) : launch_step2_bnd<false, false>(flags, a, s);
}

template <bool PML>
hipError_t launch_born_step_pml(const StepArgs &a, hipStream_t s)
{
    const dim3 grid(blocks_for(a.nwaves)), block(kLanes * kWavesPerBlock);
    if (a.dslot) {
        if (a.cw == 2) hipLaunchKernelGGL((k_born_step<2, true, PML>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_born_step<1, true, PML>), grid, block, 0, s, a);
    } else {
        if (a.cw == 2) hipLaunchKernelGGL((k_born_step<2, false, PML>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_born_step<1, false, PML>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_born_step(const StepArgs &a, hipStream_t s)
{
    if (a.nwaves <= 0) return hipSuccess;
    return a.pml ? launch_born_step_pml<true>(a, s) : launch_born_step_pml<false>(a, s);
}

hipError_t launch_scale(const float *x, float a, float *y, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_scale, dim3(unsigned(blocks)), dim3(256), 0, s, x, a, y, n);
    return hipGetLastError();
}

hipError_t launch_fill(float *p, int64_t n, float val, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill, dim3(unsigned(blocks)), dim3(256), 0, s, p, n, val);
    return hipGetLastError();
}

hipError_t launch_mute(const int64_t *off, const int32_t *nt, const float *t0, int32_t ntr, float dt, float taper,
                       const float *din, float *dout, hipStream_t s)
{
    if (ntr <= 0) return hipSuccess;
    const int blocks = ntr < 8192 ? ntr : 8192;
    hipLaunchKernelGGL(k_mute, dim3(unsigned(blocks)), dim3(256), 0, s, off, nt, t0, ntr, dt,
                       1.f / fmaxf(taper, 1e-12f), din, dout);
    return hipGetLastError();
}

hipError_t launch_laplace5(const float *x, int32_t nz, int32_t nx, float *y, hipStream_t s)
{
    const int64_t n = int64_t(nz) * nx;
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_laplace5, dim3(unsigned(blocks)), dim3(256), 0, s, x, nz, nx, y);
    return hipGetLastError();
}

hipError_t launch_model_check(const float *v, int64_t n, float *out3, hipStream_t s)
{
    hipLaunchKernelGGL(k_model_check, dim3(1), dim3(256), 0, s, v, n, out3);
    return hipGetLastError();
}

constexpr int kSumsqBlocks = 1024;   // misfit partials of the off-grid path

int64_t traces_partials_max(int32_t Q, int32_t nt_max)
{
    return std::max<int64_t>(int64_t((Q + 63) / 64) * ((nt_max + 63) / 64), kSumsqBlocks);
}

hipError_t launch_traces(const TraceArgs &a, hipStream_t s, int64_t *nblocks_out)
{
    if (!a.offgrid) {
        const unsigned gx = unsigned((a.Q + 63) / 64), gy = unsigned((a.nt_max + 63) / 64);
        if (nblocks_out) *nblocks_out = int64_t(gx) * gy;
        if (gx == 0 || gy == 0) return hipSuccess;
        hipLaunchKernelGGL(k_traces, dim3(gx, gy), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    // off the grid: receiver traces (and residuals), then the misfit and the
    // cells' adjoint sources from the residuals
    TraceArgs b = a;
    if (!a.tm_out && !a.partials) b.resid = nullptr;
    if (nblocks_out) *nblocks_out = 0;
    if (a.R > 0 && a.nt_max > 0 && (b.resid || a.tr_out)) {
        hipLaunchKernelGGL(k_traces_rec, dim3(unsigned(a.R), unsigned((a.nt_max + 255) / 256)), dim3(256), 0, s, b);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (a.partials) {
        hipLaunchKernelGGL(k_half_sumsq, dim3(kSumsqBlocks), dim3(256), 0, s, static_cast<const float *>(a.resid),
                           a.ndata, a.partials);
        if (nblocks_out) *nblocks_out = kSumsqBlocks;
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (a.tm_out && int64_t(a.nt_max) * a.Q > 0) {
        const int64_t n = int64_t(a.nt_max) * a.Q;
        hipLaunchKernelGGL(k_traces_cell, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, b);
        return hipGetLastError();
    }
    return hipSuccess;
}

hipError_t launch_sum_partials(const double *part, int64_t n, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, part, n, out);
    return hipGetLastError();
}

hipError_t launch_finalize(const FinalArgs &a, int max_nx, hipStream_t s)
{
    if (a.nshots > 0 && a.nb > 0) {
        hipLaunchKernelGGL(k_fold_rows, dim3(unsigned((max_nx + 255) / 256), unsigned(a.nshots)), dim3(256), 0, s,
                           a, max_nx);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_fold_cols, dim3(unsigned((a.nz + 255) / 256), unsigned(a.nshots)), dim3(256), 0, s, a);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int64_t n = int64_t(a.nz) * a.nx;
    hipLaunchKernelGGL(k_finalize, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace fwi
