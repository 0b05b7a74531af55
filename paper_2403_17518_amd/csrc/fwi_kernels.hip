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
// Work decomposition: a wavefront owns a 64-column strip of one shot and a
// run of rows. It streams down z keeping the nine rows of the current field
// that the vertical stencil needs in registers; the horizontal neighbours of
// the centre row go through a 72-float LDS row (64 + two 4-cell halos). The
// kernel is bound by HBM/MALL bandwidth (about 1.7 flop per byte), so no
// matrix cores are involved.
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

__device__ __forceinline__ float sponge_a(float sh)
{
    return __builtin_amdgcn_rcpf(1.0f + sh);
}

template <int FL>
__global__ __launch_bounds__(kLanes *kWavesPerBlock) void k_step(const StepArgs A)
{
    __shared__ float lds[kWavesPerBlock][kLanes + 2 * kHalo];
    const int lane = threadIdx.x & (kLanes - 1);
    const int wl = threadIdx.x / kLanes;
    const int wid = xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wl;
    if (wid >= A.nwaves) return;  // whole wave leaves; no block barrier used
    float *row = lds[wl];
    const WaveDesc W = A.waves[wid];
    const ShotDesc S = A.shots[W.shot];
    const int P = S.P;
    const int j = W.col0 + lane;
    const bool valid = j < S.NX;
    const int nb = A.nb;
    const int jm = S.x0 + clampi(j - nb, 0, S.wnx - 1);
    const int ddx = max(max(nb - j, j - (S.NX - 1 - nb)), 0);
    const float dx2 = float(ddx * ddx);
    float ax = 1.0f, bx = 1.0f;
    if (ddx > 0) {
        const float sh = A.hs * dx2;
        ax = sponge_a(sh);
        bx = (1.0f - sh) * ax;
    }
    const float *cu = A.cur + S.f_off;
    float *pv = A.prev + S.f_off;
    const int64_t goff = S.g_off;

    float q0, q1, q2, q3, q4, q5, q6, q7, q8;
    {
        const int o = (W.z0 - kHalo) * P + j;
        q0 = valid ? cu[o] : 0.0f;
        q1 = valid ? cu[o + P] : 0.0f;
        q2 = valid ? cu[o + 2 * P] : 0.0f;
        q3 = valid ? cu[o + 3 * P] : 0.0f;
        q4 = valid ? cu[o + 4 * P] : 0.0f;
        q5 = valid ? cu[o + 5 * P] : 0.0f;
        q6 = valid ? cu[o + 6 * P] : 0.0f;
        q7 = valid ? cu[o + 7 * P] : 0.0f;
    }
    int rr = W.rr0;
    int rrow = -1;
    if (FL & (F_SAMPLE | F_INJECT)) rrow = rr < W.rr1 ? A.rrows[rr].row : -1;
    const bool src_here = (FL & F_SRC) && S.src_j == j;
    const float wsrc = (FL & F_SRC) ? A.wav[S.wav_off + A.n] * A.ih2 : 0.0f;

    for (int z = W.z0; z < W.z1; ++z) {
        const int o = z * P + j;
        q8 = valid ? cu[o + kHalo * P] : 0.0f;
        row[lane + kHalo] = q4;
        if (lane < 2 * kHalo) {
            const int c = lane < kHalo ? W.col0 - kHalo + lane : W.col0 + kLanes - kHalo + lane;
            row[lane < kHalo ? lane : lane + kLanes] = (c < P) ? cu[z * P + c] : 0.0f;
        }
        wave_sync();
        float lap = A.w0 * q4 + A.w1 * ((q3 + q5) + (row[lane + 3] + row[lane + 5])) +
                    A.w2 * ((q2 + q6) + (row[lane + 2] + row[lane + 6])) +
                    A.w3 * ((q1 + q7) + (row[lane + 1] + row[lane + 7])) +
                    A.w4 * ((q0 + q8) + (row[lane] + row[lane + 8]));
        wave_sync();
        if (FL & F_SRC)
            if (src_here && z == S.src_i) lap += wsrc;
        int qi = -1;
        if (FL & (F_SAMPLE | F_INJECT)) {
            if (z == rrow) {
                qi = A.rmap[A.rrows[rr].map_off + lane];
                ++rr;
                rrow = rr < W.rr1 ? A.rrows[rr].row : -1;
            }
            if (FL & F_INJECT)
                if (qi >= 0) lap += A.inj[qi];
        }
        const float V = A.v[clampi(z - nb, 0, A.nz - 1) * A.nx + jm];
        const float c = V * V * A.dt2;
        float a = ax, b = bx;
        const int ddz = max(max(nb - z, z - (A.NZ - 1 - nb)), 0);
        if (ddz > 0) {
            const float sh = A.hs * (float(ddz * ddz) + dx2);
            a = sponge_a(sh);
            b = (1.0f - sh) * a;
        }
        const float D = c * lap;
        if (valid) {
            const float out = a * (2.0f * q4 + D) - b * pv[o];
            pv[o] = out;
            if (FL & F_EMIT) A.dslot[goff + o] = D;
            if (FL & F_IMAGE) A.G[goff + o] += out * A.dslot[goff + o];
            if (FL & F_SAMPLE)
                if (qi >= 0) A.samp[qi] = out;
        }
        q0 = q1; q1 = q2; q2 = q3; q3 = q4; q4 = q5; q5 = q6; q6 = q7; q7 = q8;
    }
}

// Born: background u and scattered du advanced together (section 2.2: the
// two equations are solved jointly so that u is never stored):
//   du^{n+1} = a (2 du^n + V^2 dt^2 L8 du^n + 2 V dV dt^2 (L8 u^n + s^n)) - b du^{n-1}
// where 2 V dV dt^2 = (2 dV / V) V^2 dt^2 is the linearised 1/V^2 term.
__global__ __launch_bounds__(kLanes *kWavesPerBlock) void k_born_step(const StepArgs A)
{
    __shared__ float lds[kWavesPerBlock][2][kLanes + 2 * kHalo];
    const int lane = threadIdx.x & (kLanes - 1);
    const int wl = threadIdx.x / kLanes;
    const int wid = xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wl;
    if (wid >= A.nwaves) return;
    float *row = lds[wl][0];
    float *rod = lds[wl][1];
    const WaveDesc W = A.waves[wid];
    const ShotDesc S = A.shots[W.shot];
    const int P = S.P;
    const int j = W.col0 + lane;
    const bool valid = j < S.NX;
    const int nb = A.nb;
    const int jm = S.x0 + clampi(j - nb, 0, S.wnx - 1);
    const int ddx = max(max(nb - j, j - (S.NX - 1 - nb)), 0);
    const float dx2 = float(ddx * ddx);
    float ax = 1.0f, bx = 1.0f;
    if (ddx > 0) {
        const float sh = A.hs * dx2;
        ax = sponge_a(sh);
        bx = (1.0f - sh) * ax;
    }
    const float *cu = A.cur + S.f_off;
    float *pv = A.prev + S.f_off;
    const float *cd = A.cur2 + S.f_off;
    float *pd = A.prev2 + S.f_off;

    float q[9], r[9];
    {
        const int o = (W.z0 - kHalo) * P + j;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            q[k] = valid ? cu[o + k * P] : 0.0f;
            r[k] = valid ? cd[o + k * P] : 0.0f;
        }
    }
    int rr = W.rr0;
    int rrow = rr < W.rr1 ? A.rrows[rr].row : -1;
    const bool src_here = S.src_j == j;
    const float wsrc = A.wav[S.wav_off + A.n] * A.ih2;

    for (int z = W.z0; z < W.z1; ++z) {
        const int o = z * P + j;
        q[8] = valid ? cu[o + kHalo * P] : 0.0f;
        r[8] = valid ? cd[o + kHalo * P] : 0.0f;
        row[lane + kHalo] = q[4];
        rod[lane + kHalo] = r[4];
        if (lane < 2 * kHalo) {
            const int c = lane < kHalo ? W.col0 - kHalo + lane : W.col0 + kLanes - kHalo + lane;
            const int li = lane < kHalo ? lane : lane + kLanes;
            row[li] = (c < P) ? cu[z * P + c] : 0.0f;
            rod[li] = (c < P) ? cd[z * P + c] : 0.0f;
        }
        wave_sync();
        float lap = A.w0 * q[4] + A.w1 * ((q[3] + q[5]) + (row[lane + 3] + row[lane + 5])) +
                    A.w2 * ((q[2] + q[6]) + (row[lane + 2] + row[lane + 6])) +
                    A.w3 * ((q[1] + q[7]) + (row[lane + 1] + row[lane + 7])) +
                    A.w4 * ((q[0] + q[8]) + (row[lane] + row[lane + 8]));
        const float lapd = A.w0 * r[4] + A.w1 * ((r[3] + r[5]) + (rod[lane + 3] + rod[lane + 5])) +
                           A.w2 * ((r[2] + r[6]) + (rod[lane + 2] + rod[lane + 6])) +
                           A.w3 * ((r[1] + r[7]) + (rod[lane + 1] + rod[lane + 7])) +
                           A.w4 * ((r[0] + r[8]) + (rod[lane] + rod[lane + 8]));
        wave_sync();
        if (src_here && z == S.src_i) lap += wsrc;
        int qi = -1;
        if (z == rrow) {
            qi = A.rmap[A.rrows[rr].map_off + lane];
            ++rr;
            rrow = rr < W.rr1 ? A.rrows[rr].row : -1;
        }
        const int mi = clampi(z - nb, 0, A.nz - 1) * A.nx + jm;
        const float V = A.v[mi];
        const float dV = A.dv[mi];
        const float c = V * V * A.dt2;
        const float cr = 2.0f * V * dV * A.dt2;
        float a = ax, b = bx;
        const int ddz = max(max(nb - z, z - (A.NZ - 1 - nb)), 0);
        if (ddz > 0) {
            const float sh = A.hs * (float(ddz * ddz) + dx2);
            a = sponge_a(sh);
            b = (1.0f - sh) * a;
        }
        if (valid) {
            const float ou = a * (2.0f * q[4] + c * lap) - b * pv[o];
            const float od = a * (2.0f * r[4] + c * lapd + cr * lap) - b * pd[o];
            pv[o] = ou;
            pd[o] = od;
            if (qi >= 0) A.samp[qi] = od;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            q[k] = q[k + 1];
            r[k] = r[k + 1];
        }
    }
}

__global__ void k_fill(float *p, int64_t n, float val)
{
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = val;
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

// img = (2 / (v^3 dt^2)) sum_shots Pad^T G_s. Pad^T folds every sponge cell
// onto the edge cell whose value it replicates; shots are summed in slot
// order, so the result does not depend on scheduling.
__global__ __launch_bounds__(256) void k_finalize(const FinalArgs A)
{
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= int64_t(A.nz) * A.nx) return;
    const int i = int(p / A.nx), j = int(p % A.nx);
    const int nb = A.nb;
    const int r0 = i == 0 ? 0 : i + nb;
    const int r1 = i == A.nz - 1 ? A.NZ - 1 : i + nb;
    float acc = 0.0f;
    for (int s = 0; s < A.nshots; ++s) {
        const ShotDesc S = A.shots[s];
        const int jl = j - S.x0;
        if (jl < 0 || jl >= S.wnx) continue;
        const int c0 = jl == 0 ? 0 : jl + nb;
        const int c1 = jl == S.wnx - 1 ? S.NX - 1 : jl + nb;
        const float *G = A.G + S.g_off;
        for (int r = r0; r <= r1; ++r)
            for (int c = c0; c <= c1; ++c) acc += G[int64_t(r) * S.P + c];
    }
    const float v = A.v[p];
    A.img[p] = acc * (2.0f / (v * v * v * A.dt2));
}

inline int blocks_for(int nwaves) { return (nwaves + kWavesPerBlock - 1) / kWavesPerBlock; }

}  // namespace

hipError_t launch_step(int flags, const StepArgs &a, hipStream_t s)
{
    if (a.nwaves <= 0) return hipSuccess;
    const dim3 grid(blocks_for(a.nwaves)), block(kLanes * kWavesPerBlock);
    switch (flags) {
    case F_SRC | F_SAMPLE:
        hipLaunchKernelGGL(k_step<F_SRC | F_SAMPLE>, grid, block, 0, s, a);
        break;
    case F_SRC:
        hipLaunchKernelGGL(k_step<F_SRC>, grid, block, 0, s, a);
        break;
    case F_SRC | F_SAMPLE | F_EMIT:
        hipLaunchKernelGGL(k_step<F_SRC | F_SAMPLE | F_EMIT>, grid, block, 0, s, a);
        break;
    case F_SRC | F_EMIT:
        hipLaunchKernelGGL(k_step<F_SRC | F_EMIT>, grid, block, 0, s, a);
        break;
    case F_INJECT | F_IMAGE:
        hipLaunchKernelGGL(k_step<F_INJECT | F_IMAGE>, grid, block, 0, s, a);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_born_step(const StepArgs &a, hipStream_t s)
{
    if (a.nwaves <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_born_step, dim3(blocks_for(a.nwaves)), dim3(kLanes * kWavesPerBlock), 0, s, a);
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

hipError_t launch_model_check(const float *v, int64_t n, float *out3, hipStream_t s)
{
    hipLaunchKernelGGL(k_model_check, dim3(1), dim3(256), 0, s, v, n, out3);
    return hipGetLastError();
}

hipError_t launch_traces(const TraceArgs &a, hipStream_t s, int64_t *nblocks_out)
{
    const unsigned gx = unsigned((a.Q + 63) / 64), gy = unsigned((a.nt_max + 63) / 64);
    if (nblocks_out) *nblocks_out = int64_t(gx) * gy;
    if (gx == 0 || gy == 0) return hipSuccess;
    hipLaunchKernelGGL(k_traces, dim3(gx, gy), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double *part, int64_t n, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, part, n, out);
    return hipGetLastError();
}

hipError_t launch_finalize(const FinalArgs &a, hipStream_t s)
{
    const int64_t n = int64_t(a.nz) * a.nx;
    hipLaunchKernelGGL(k_finalize, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace fwi
