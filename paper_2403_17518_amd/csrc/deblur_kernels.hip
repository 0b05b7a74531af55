// HIP kernels (gfx950) of the deblurring network that approximates the
// inverse Hessian (paper section 2.3: a UNet-like network trained to map the
// doubly migrated image to the FWI gradient; architecture in Appendix A,
// Table 1).
//
// Convolutions are implicit GEMMs on the bf16 matrix cores
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation): a workgroup of 4 waves owns a
// (32*WM) x (32*WN) output tile, stages 32-deep K slices of the weight matrix
// and of the gathered activations in LDS, and each wave accumulates one 32x32
// block. The same kernel runs the forward 3x3 convolutions, their data
// gradients (with flipped, transposed weights), the 2x2 stride-2 transposed
// convolutions (scatter epilogue) and their data gradients (stride-2 gather).
// Weight gradients reduce over pixels in a second kernel, split over pixel
// chunks with a deterministic reduction of the partial sums.
#include "deblur_internal.h"

namespace dbl {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kBK = 32;
constexpr int kLDK = kBK + 8;  // LDS row stride (bf16): 80 B, 16-B aligned

__device__ __forceinline__ float bf2f(bf16 x) { return float(x); }
__device__ __forceinline__ bf16 f2bf(float x) { return bf16(x); }

// gathered source pixel index, or -1 outside the source grid
__device__ __forceinline__ int64_t gather_pix(const Gather &g, int p, int tap)
{
    const int i = p / g.W, j = p - (p / g.W) * g.W;
    const int si = i * g.stride + tap / g.tapw + g.d0;
    const int sj = j * g.stride + tap % g.tapw + g.d0;
    if (si < 0 || si >= g.Hs || sj < 0 || sj >= g.Ws) return -1;
    return int64_t(si) * g.Ws + sj;
}

template <int WM, int WN, int TN, bool VEC>
__global__ __launch_bounds__(256) void k_gemm(const GemmArgs a)
{
    // each wave accumulates a 32 x (32*TN) block: TN matrix-core tiles share
    // one A operand per K slice
    constexpr int BM = 32 * WM, BN = 32 * WN * TN;
    __shared__ __attribute__((aligned(16))) bf16 As[BM * kLDK];
    __shared__ __attribute__((aligned(16))) bf16 Bs[BN * kLDK];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w / WN, wn = w % WN;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int nk = (a.K + kBK - 1) / kBK;
    const Gather &g = a.g;

    constexpr int ACH = BM * kBK / 8, BCH = BN * kBK / 8;   // 16-byte chunks per tile
    constexpr int AR = (ACH + 255) / 256, BR = (BCH + 255) / 256;
    uint4 ra[AR], rb[BR];
    // scalar staging for the generic path
    constexpr int AE = (BM * kBK + 255) / 256, BE = (BN * kBK + 255) / 256;
    bf16 sa[VEC ? 1 : AE], sb[VEC ? 1 : BE];

    auto load_tiles = [&](int kt) {
        const int kbase = kt * kBK;
        if constexpr (VEC) {
#pragma unroll
            for (int r = 0; r < AR; ++r) {
                const int c = tid + r * 256;
                uint4 v = make_uint4(0, 0, 0, 0);
                if (c < ACH) {
                    const int row = c / 4, kc = (c % 4) * 8;
                    if (m0 + row < a.M)
                        v = *reinterpret_cast<const uint4 *>(a.A + int64_t(m0 + row) * a.lda + kbase + kc);
                }
                ra[r] = v;
            }
#pragma unroll
            for (int r = 0; r < BR; ++r) {
                const int c = tid + r * 256;
                uint4 v = make_uint4(0, 0, 0, 0);
                if (c < BCH) {
                    const int nl = c / 4, kc = (c % 4) * 8;
                    const int p = n0 + nl;
                    const int k = kbase + kc;
                    if (p < a.N) {
                        const int tap = k / g.Cb, ch = k - tap * g.Cb;
                        const int64_t sp = gather_pix(g, p, tap);
                        if (sp >= 0) v = *reinterpret_cast<const uint4 *>(g.src + sp * g.ld + g.coff + ch);
                    }
                }
                rb[r] = v;
            }
        } else {
#pragma unroll
            for (int r = 0; r < AE; ++r) {
                const int e = tid + r * 256;
                bf16 v = f2bf(0.f);
                if (e < BM * kBK) {
                    const int row = e / kBK, k = kbase + e % kBK;
                    if (m0 + row < a.M && k < a.K) v = a.A[int64_t(m0 + row) * a.lda + k];
                }
                sa[r] = v;
            }
#pragma unroll
            for (int r = 0; r < BE; ++r) {
                const int e = tid + r * 256;
                bf16 v = f2bf(0.f);
                if (e < BN * kBK) {
                    const int nl = e / kBK, k = kbase + e % kBK;
                    const int p = n0 + nl;
                    if (p < a.N && k < a.K) {
                        const int tap = k / g.Cb, ch = k - tap * g.Cb;
                        const int64_t sp = gather_pix(g, p, tap);
                        if (sp >= 0) v = g.src[sp * g.ld + g.coff + ch];
                    }
                }
                sb[r] = v;
            }
        }
    };
    auto store_tiles = [&]() {
        if constexpr (VEC) {
#pragma unroll
            for (int r = 0; r < AR; ++r) {
                const int c = tid + r * 256;
                if (c < ACH) *reinterpret_cast<uint4 *>(&As[(c / 4) * kLDK + (c % 4) * 8]) = ra[r];
            }
#pragma unroll
            for (int r = 0; r < BR; ++r) {
                const int c = tid + r * 256;
                if (c < BCH) *reinterpret_cast<uint4 *>(&Bs[(c / 4) * kLDK + (c % 4) * 8]) = rb[r];
            }
        } else {
#pragma unroll
            for (int r = 0; r < AE; ++r) {
                const int e = tid + r * 256;
                if (e < BM * kBK) As[(e / kBK) * kLDK + e % kBK] = sa[r];
            }
#pragma unroll
            for (int r = 0; r < BE; ++r) {
                const int e = tid + r * 256;
                if (e < BN * kBK) Bs[(e / kBK) * kLDK + e % kBK] = sb[r];
            }
        }
    };

    f32x16 acc[TN];
#pragma unroll
    for (int tn = 0; tn < TN; ++tn) acc[tn] = f32x16{};
    load_tiles(0);
    for (int kt = 0; kt < nk; ++kt) {
        __syncthreads();
        store_tiles();
        __syncthreads();
        if (kt + 1 < nk) load_tiles(kt + 1);
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const bf16x8 av =
                *reinterpret_cast<const bf16x8 *>(&As[(wm * 32 + lane % 32) * kLDK + kk * 16 + 8 * (lane / 32)]);
#pragma unroll
            for (int tn = 0; tn < TN; ++tn) {
                const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(
                    &Bs[((wn * TN + tn) * 32 + lane % 32) * kLDK + kk * 16 + 8 * (lane / 32)]);
                acc[tn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[tn], 0, 0, 0);
            }
        }
    }
    // epilogue: lane holds rows m = 8*(i/4) + 4*(lane/32) + i%4, column lane%32
#pragma unroll
    for (int tn = 0; tn < TN; ++tn) {
        const int n = n0 + (wn * TN + tn) * 32 + lane % 32;
        if (n >= a.N) continue;
        const int pi = n / g.W, pj = n - (n / g.W) * g.W;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int m = m0 + wm * 32 + 8 * (i / 4) + 4 * (lane / 32) + (i % 4);
            if (m >= a.M) continue;
            int co = m;
            int64_t pix = n;
            if (a.scatter) {
                const int ab = m / a.Cout;
                co = m - ab * a.Cout;
                pix = int64_t(2 * pi + ab / 2) * a.Wo + 2 * pj + ab % 2;
            }
            float v = acc[tn][i];
            if (a.bias) v += a.bias[co];
            if (a.act) v = v > 0.f ? v : a.slope * v;
            if (a.act_y && !(bf2f(a.act_y[pix * a.act_ld + a.act_coff + co]) > 0.f)) v *= a.slope;
            a.out[pix * a.out_ld + a.out_coff + co] = f2bf(v);
        }
    }
}

// Epilogue of one 32 x 32 accumulator tile of the implicit GEMMs with
// vectorised outputs (out_vec): the lane holds channels m = mt + 8 j +
// 4 (lane / 32) + q (j, q < 4) of output column n, so the four consecutive
// channels of each j leave as one 8-byte store (and the activation
// derivative, if any, arrives as one 8-byte load).
__device__ __forceinline__ void gemm_store_tile(const GemmArgs &a, const f32x16 &acc, int mt, int n, int lane)
{
    if (n >= a.N) return;
    const int pi = n / a.g.W, pj = n - (n / a.g.W) * a.g.W;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int mb = mt + 8 * j + 4 * (lane / 32);
        if (mb >= a.M) continue;
        int co = mb;
        int64_t pix = n;
        if (a.scatter) {
            const int ab = mb / a.Cout;
            co = mb - ab * a.Cout;
            pix = int64_t(2 * pi + ab / 2) * a.Wo + 2 * pj + ab % 2;
        }
        float v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v[q] = acc[4 * j + q];
            if (a.bias) v[q] += a.bias[co + q];
            if (a.act) v[q] = v[q] > 0.f ? v[q] : a.slope * v[q];
        }
        if (a.act_y) {
            const uint2 yw = *reinterpret_cast<const uint2 *>(a.act_y + pix * a.act_ld + a.act_coff + co);
            const bf16 *y = reinterpret_cast<const bf16 *>(&yw);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (!(bf2f(y[q]) > 0.f)) v[q] *= a.slope;
        }
        bf16 o[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) o[q] = f2bf(v[q]);
        *reinterpret_cast<uint2 *>(a.out + pix * a.out_ld + a.out_coff + co) = *reinterpret_cast<const uint2 *>(o);
    }
}

// Implicit GEMM with 16-byte operand loads: a (32*WM) x (32*WN*TN) output
// tile per workgroup, 32-deep K slices double-buffered in LDS (one barrier
// per slice). The output pixels whose gathered rows a thread loads are the
// same in every slice, so their coordinates are computed once, and the tap
// and channel of each row's K offset advance with the slice instead of being
// divided out at every load; the loads of the next DEPTH slices are in
// flight while a slice is computed (a ring of register stages). Requires K,
// Cb, lda, ld and coff to be multiples of 8 and K a multiple of 32. Same
// epilogue as k_gemm.
template <int WM, int WN, int TN, int DEPTH>
__global__ __launch_bounds__(256) void k_gemm_v(const GemmArgs a)
{
    constexpr int BM = 32 * WM, BN = 32 * WN * TN;
    __shared__ __attribute__((aligned(16))) bf16 As[2][BM * kLDK];
    __shared__ __attribute__((aligned(16))) bf16 Bs[2][BN * kLDK];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w / WN, wn = w % WN;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int nk = a.K / kBK;
    const Gather &g = a.g;
    constexpr int ACH = BM * kBK / 8, BCH = BN * kBK / 8;   // 16-byte chunks per tile
    constexpr int AR = (ACH + 255) / 256, BR = (BCH + 255) / 256;
    // the thread's B rows: pixel coordinates, and the running tap (ty, tx)
    // and channel of the row's 8-wide K offset
    int bpi[BR], bpj[BR], bch[BR], bty[BR], btx[BR];
    bool bok[BR];
#pragma unroll
    for (int r = 0; r < BR; ++r) {
        const int c = tid + r * 256, p = n0 + (c >> 2), kc = (c & 3) * 8;
        bok[r] = c < BCH && p < a.N;
        bpi[r] = bok[r] ? p / g.W : 0;
        bpj[r] = bok[r] ? p - bpi[r] * g.W : 0;
        const int tap = kc / g.Cb;
        bch[r] = kc - tap * g.Cb;
        bty[r] = tap / g.tapw;
        btx[r] = tap - bty[r] * g.tapw;
    }
    uint4 ra[DEPTH][AR], rb[DEPTH][BR];
    auto load = [&](int kt, int sl) {
        const int kbase = kt * kBK;
#pragma unroll
        for (int r = 0; r < AR; ++r) {
            const int c = tid + r * 256;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (c < ACH && m0 + (c >> 2) < a.M)
                v = *reinterpret_cast<const uint4 *>(a.A + int64_t(m0 + (c >> 2)) * a.lda + kbase + (c & 3) * 8);
            ra[sl][r] = v;
        }
#pragma unroll
        for (int r = 0; r < BR; ++r) {
            uint4 v = make_uint4(0, 0, 0, 0);
            if (bok[r]) {
                const int si = bpi[r] * g.stride + bty[r] + g.d0, sj = bpj[r] * g.stride + btx[r] + g.d0;
                if (si >= 0 && si < g.Hs && sj >= 0 && sj < g.Ws)
                    v = *reinterpret_cast<const uint4 *>(g.src + (int64_t(si) * g.Ws + sj) * g.ld + g.coff + bch[r]);
            }
            rb[sl][r] = v;
        }
    };
    auto advance = [&]() {   // the K offsets move on by one slice
#pragma unroll
        for (int r = 0; r < BR; ++r) {
            bch[r] += kBK;
            while (bch[r] >= g.Cb) {
                bch[r] -= g.Cb;
                if (++btx[r] == g.tapw) {
                    btx[r] = 0;
                    ++bty[r];
                }
            }
        }
    };
    auto store = [&](int sl, int buf) {
#pragma unroll
        for (int r = 0; r < AR; ++r) {
            const int c = tid + r * 256;
            if (c < ACH) *reinterpret_cast<uint4 *>(&As[buf][(c >> 2) * kLDK + (c & 3) * 8]) = ra[sl][r];
        }
#pragma unroll
        for (int r = 0; r < BR; ++r) {
            const int c = tid + r * 256;
            if (c < BCH) *reinterpret_cast<uint4 *>(&Bs[buf][(c >> 2) * kLDK + (c & 3) * 8]) = rb[sl][r];
        }
    };

    f32x16 acc[TN];
#pragma unroll
    for (int tn = 0; tn < TN; ++tn) acc[tn] = f32x16{};
    // ring of register stages as in k_wgrad_t (the tap state advances in
    // load order)
#pragma unroll
    for (int d = 0; d < DEPTH; ++d)
        if (d < nk) {
            load(d, d);
            advance();
        }
    if (nk > 0) store(0, 0);
    __syncthreads();
    for (int kt0 = 0; kt0 < nk; kt0 += DEPTH) {
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) {
            const int kt = kt0 + d;
            if (kt < nk) {
                const int buf = kt & 1;
                if (kt + DEPTH < nk) {
                    load(kt + DEPTH, d);
                    advance();
                }
#pragma unroll
                for (int kk = 0; kk < 2; ++kk) {
                    const bf16x8 av = *reinterpret_cast<const bf16x8 *>(
                        &As[buf][(wm * 32 + lane % 32) * kLDK + kk * 16 + 8 * (lane / 32)]);
#pragma unroll
                    for (int tn = 0; tn < TN; ++tn) {
                        const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(
                            &Bs[buf][((wn * TN + tn) * 32 + lane % 32) * kLDK + kk * 16 + 8 * (lane / 32)]);
                        acc[tn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[tn], 0, 0, 0);
                    }
                }
                if (kt + 1 < nk) store((d + 1) % DEPTH, buf ^ 1);
                __syncthreads();
            }
        }
    }
    // epilogue: lane holds rows m = 8*(i/4) + 4*(lane/32) + i%4, column lane%32
#pragma unroll
    for (int tn = 0; tn < TN; ++tn) {
        const int n = n0 + (wn * TN + tn) * 32 + lane % 32;
        if (a.out_vec) {
            gemm_store_tile(a, acc[tn], m0 + wm * 32, n, lane);
            continue;
        }
        if (n >= a.N) continue;
        const int pi = n / g.W, pj = n - (n / g.W) * g.W;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int m = m0 + wm * 32 + 8 * (i / 4) + 4 * (lane / 32) + (i % 4);
            if (m >= a.M) continue;
            int co = m;
            int64_t pix = n;
            if (a.scatter) {
                const int ab = m / a.Cout;
                co = m - ab * a.Cout;
                pix = int64_t(2 * pi + ab / 2) * a.Wo + 2 * pj + ab % 2;
            }
            float v = acc[tn][i];
            if (a.bias) v += a.bias[co];
            if (a.act) v = v > 0.f ? v : a.slope * v;
            if (a.act_y && !(bf2f(a.act_y[pix * a.act_ld + a.act_coff + co]) > 0.f)) v *= a.slope;
            a.out[pix * a.out_ld + a.out_coff + co] = f2bf(v);
        }
    }
}

// Implicit GEMM for wide layers: a 128 x 128 output tile per workgroup (4
// waves of 64 x 64, four 32 x 32 matrix-core tiles each), 64-deep K slices
// staged through registers into LDS. Each thread loads 4 rows of A and 4
// gathered rows of B at one 8-element K offset; the tap and channel of that
// offset are computed once per slice and the pixel coordinates of the rows
// once per kernel. Requires K, Cb, lda, ld and coff to be multiples of 8 and
// K a multiple of 64. Same epilogue as k_gemm.
__global__ __launch_bounds__(256) void k_gemm2(const GemmArgs a)
{
    constexpr int BM = 128, BN = 128, BK = 64, LDK = BK + 8;
    __shared__ __attribute__((aligned(16))) bf16 As[BM * LDK];
    __shared__ __attribute__((aligned(16))) bf16 Bs[BN * LDK];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const Gather &g = a.g;
    // split K: workgroup z takes slices [z*nkz, (z+1)*nkz)
    const int nkz = (a.K / BK + gridDim.z - 1) / gridDim.z;
    const int kt0 = blockIdx.z * nkz;
    const int nk = max(0, min(a.K / BK, kt0 + nkz) - kt0);
    const int kc = (tid & 7) * 8;     // this thread's K offset within a slice
    const int r0 = tid >> 3;          // rows r0, r0 + 32, r0 + 64, r0 + 96
    int pi[4], pj[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int p = n0 + r0 + 32 * u;
        pi[u] = p < a.N ? p / g.W : -1 << 20;   // rows past N never pass the bounds test
        pj[u] = p < a.N ? p - (p / g.W) * g.W : 0;
    }
    uint4 ra[4], rb[4];
    auto load = [&](int kt) {
        const int k = (kt0 + kt) * BK + kc;
        const int tap = k / g.Cb, ch = k - (k / g.Cb) * g.Cb;
        const int ty = tap / g.tapw, tx = tap - (tap / g.tapw) * g.tapw;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int m = m0 + r0 + 32 * u;
            ra[u] = m < a.M ? *reinterpret_cast<const uint4 *>(a.A + int64_t(m) * a.lda + k) : make_uint4(0, 0, 0, 0);
            const int si = pi[u] * g.stride + ty + g.d0, sj = pj[u] * g.stride + tx + g.d0;
            rb[u] = (si >= 0 && si < g.Hs && sj >= 0 && sj < g.Ws)
                        ? *reinterpret_cast<const uint4 *>(g.src + (int64_t(si) * g.Ws + sj) * g.ld + g.coff + ch)
                        : make_uint4(0, 0, 0, 0);
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            *reinterpret_cast<uint4 *>(&As[(r0 + 32 * u) * LDK + kc]) = ra[u];
            *reinterpret_cast<uint4 *>(&Bs[(r0 + 32 * u) * LDK + kc]) = rb[u];
        }
    };
    f32x16 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = f32x16{};
    if (nk > 0) load(0);
    for (int kt = 0; kt < nk; ++kt) {
        __syncthreads();
        store();
        __syncthreads();
        if (kt + 1 < nk) load(kt + 1);
#pragma unroll
        for (int kk = 0; kk < BK / 16; ++kk) {
            bf16x8 av[2], bv[2];
#pragma unroll
            for (int x = 0; x < 2; ++x)
                av[x] = *reinterpret_cast<const bf16x8 *>(
                    &As[(wm * 64 + x * 32 + lane % 32) * LDK + kk * 16 + 8 * (lane / 32)]);
#pragma unroll
            for (int y = 0; y < 2; ++y)
                bv[y] = *reinterpret_cast<const bf16x8 *>(
                    &Bs[(wn * 64 + y * 32 + lane % 32) * LDK + kk * 16 + 8 * (lane / 32)]);
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[x], bv[y], acc[x][y], 0, 0, 0);
        }
    }
    if (gridDim.z > 1) {
        // split K: raw partial sums, [z][n][m]
        float *part = a.kpart + int64_t(blockIdx.z) * a.N * a.M;
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int n = n0 + wn * 64 + y * 32 + lane % 32;
            if (n >= a.N) continue;
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int mb = m0 + wm * 64 + x * 32 + 8 * j + 4 * (lane / 32);
                    if (mb >= a.M) continue;
                    if (a.out_vec) {
                        *reinterpret_cast<float4 *>(part + int64_t(n) * a.M + mb) =
                            make_float4(acc[x][y][4 * j], acc[x][y][4 * j + 1], acc[x][y][4 * j + 2],
                                        acc[x][y][4 * j + 3]);
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if (mb + q < a.M) part[int64_t(n) * a.M + mb + q] = acc[x][y][4 * j + q];
                    }
                }
        }
        return;
    }
    // epilogue: lane holds rows m = 8*(i/4) + 4*(lane/32) + i%4 of each tile, column lane%32
    if (a.out_vec) {
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int x = 0; x < 2; ++x)
                gemm_store_tile(a, acc[x][y], m0 + wm * 64 + x * 32, n0 + wn * 64 + y * 32 + lane % 32, lane);
        return;
    }
#pragma unroll
    for (int y = 0; y < 2; ++y) {
        const int n = n0 + wn * 64 + y * 32 + lane % 32;
        if (n >= a.N) continue;
        const int pi_ = n / g.W, pj_ = n - (n / g.W) * g.W;
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int m = m0 + wm * 64 + x * 32 + 8 * (i / 4) + 4 * (lane / 32) + (i % 4);
                if (m >= a.M) continue;
                int co = m;
                int64_t pix = n;
                if (a.scatter) {
                    const int ab = m / a.Cout;
                    co = m - ab * a.Cout;
                    pix = int64_t(2 * pi_ + ab / 2) * a.Wo + 2 * pj_ + ab % 2;
                }
                float v = acc[x][y][i];
                if (a.bias) v += a.bias[co];
                if (a.act) v = v > 0.f ? v : a.slope * v;
                if (a.act_y && !(bf2f(a.act_y[pix * a.act_ld + a.act_coff + co]) > 0.f)) v *= a.slope;
                a.out[pix * a.out_ld + a.out_coff + co] = f2bf(v);
            }
    }
}

template <bool VEC>
__global__ __launch_bounds__(256) void k_wgrad(const WgradArgs a)
{
    constexpr int BM = 64, BN = 64;
    __shared__ __attribute__((aligned(16))) bf16 As[BM * kLDK];
    __shared__ __attribute__((aligned(16))) bf16 Bs[BN * kLDK];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w / 2, wn = w % 2;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const Gather &g = a.g;
    const int P = g.H * g.W;
    const int p_lo = blockIdx.z * a.chunk;
    const int p_hi = min(P, p_lo + a.chunk);
    const int nk = p_hi > p_lo ? (p_hi - p_lo + kBK - 1) / kBK : 0;

    // VEC: each thread moves one 8-wide chunk of A (8 m values of one pixel)
    // and one of B (8 n values of one pixel); LDS tiles are [m][pixel] and
    // [n][pixel] so the matrix-core operands read 8 consecutive pixels.
    uint4 ra = make_uint4(0, 0, 0, 0), rb = make_uint4(0, 0, 0, 0);
    bf16 sa[8], sb[8];
    int pl = 0, mc = 0;
    auto load_tiles = [&](int kt) {
        const int pbase = p_lo + kt * kBK;
        if constexpr (VEC) {
            pl = tid / 8;
            mc = (tid % 8) * 8;
            const int p = pbase + pl;
            ra = make_uint4(0, 0, 0, 0);
            rb = make_uint4(0, 0, 0, 0);
            if (p < p_hi) {
                if (m0 + mc < a.M) ra = *reinterpret_cast<const uint4 *>(a.A + int64_t(p) * a.lda + a.acoff + m0 + mc);
                const int nn = n0 + mc;
                if (nn < a.N) {
                    const int tap = nn / g.Cb, ch = nn - tap * g.Cb;
                    const int64_t sp = gather_pix(g, p, tap);
                    if (sp >= 0) rb = *reinterpret_cast<const uint4 *>(g.src + sp * g.ld + g.coff + ch);
                }
            }
        } else {
            pl = tid / 8;
            mc = (tid % 8) * 8;
            const int p = pbase + pl;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                bf16 va = f2bf(0.f), vb = f2bf(0.f);
                if (p < p_hi) {
                    if (m0 + mc + e < a.M) va = a.A[int64_t(p) * a.lda + a.acoff + m0 + mc + e];
                    const int nn = n0 + mc + e;
                    if (nn < a.N) {
                        const int tap = nn / g.Cb, ch = nn - tap * g.Cb;
                        const int64_t sp = gather_pix(g, p, tap);
                        if (sp >= 0) vb = g.src[sp * g.ld + g.coff + ch];
                    }
                }
                sa[e] = va;
                sb[e] = vb;
            }
        }
    };
    auto store_tiles = [&]() {
        if constexpr (VEC) {
            const bf16 *pa = reinterpret_cast<const bf16 *>(&ra);
            const bf16 *pb = reinterpret_cast<const bf16 *>(&rb);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                As[(mc + e) * kLDK + pl] = pa[e];
                Bs[(mc + e) * kLDK + pl] = pb[e];
            }
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                As[(mc + e) * kLDK + pl] = sa[e];
                Bs[(mc + e) * kLDK + pl] = sb[e];
            }
        }
    };

    // the first column of blocks also sums A over its pixels: the bias
    // gradient of the layer (A = dz), per split, reduced later in order
    const bool do_bias = a.bias_partial != nullptr && blockIdx.x == 0;
    float bsum[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    f32x16 acc = {};
    if (nk > 0) load_tiles(0);
    for (int kt = 0; kt < nk; ++kt) {
        __syncthreads();
        store_tiles();
        if (do_bias) {
            if constexpr (VEC) {
                const bf16 *pa = reinterpret_cast<const bf16 *>(&ra);
#pragma unroll
                for (int e = 0; e < 8; ++e) bsum[e] += bf2f(pa[e]);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) bsum[e] += bf2f(sa[e]);
            }
        }
        __syncthreads();
        if (kt + 1 < nk) load_tiles(kt + 1);
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const bf16x8 av =
                *reinterpret_cast<const bf16x8 *>(&As[(wm * 32 + lane % 32) * kLDK + kk * 16 + 8 * (lane / 32)]);
            const bf16x8 bv =
                *reinterpret_cast<const bf16x8 *>(&Bs[(wn * 32 + lane % 32) * kLDK + kk * 16 + 8 * (lane / 32)]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
        }
    }
    if (do_bias) {
        // threads tid, tid+8, ... hold the same 8 channels for 32 pixel rows
        __shared__ float bred[32][65];
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 8; ++e) bred[tid / 8][(tid % 8) * 8 + e] = bsum[e];
        __syncthreads();
        if (tid < 64) {
            float t = 0.f;
            for (int r = 0; r < 32; ++r) t += bred[r][tid];
            if (m0 + tid < a.M) a.bias_partial[int64_t(blockIdx.z) * a.M + m0 + tid] = t;
        }
    }
    const int n = n0 + wn * 32 + lane % 32;
    if (n >= a.N) return;
    float *part = a.partial + int64_t(blockIdx.z) * a.M * a.N;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int m = m0 + wm * 32 + 8 * (i / 4) + 4 * (lane / 32) + (i % 4);
        if (m < a.M) part[int64_t(m) * a.N + n] = acc[i];
    }
}

// sum of `rows` partial rows with four independent accumulators (the loads
// of a thread overlap; the combination order is fixed)
__device__ __forceinline__ float sum_strided(const float *p, int rows, int64_t stride)
{
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    int z = 0;
    for (; z + 4 <= rows; z += 4) {
        s0 += p[int64_t(z) * stride];
        s1 += p[int64_t(z + 1) * stride];
        s2 += p[int64_t(z + 2) * stride];
        s3 += p[int64_t(z + 3) * stride];
    }
    for (; z < rows; ++z) s0 += p[int64_t(z) * stride];
    return (s0 + s1) + (s2 + s3);
}

// split-K second pass: sums the parts of output (m, n) in order, then bias,
// activation and the bf16 store (or scatter) of the GEMM epilogue
__global__ void k_gemm_finish(const GemmArgs a, int32_t ksplit)
{
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= int64_t(a.M) * a.N) return;
    const int m = int(e % a.M), n = int(e / a.M);
    float v = sum_strided(a.kpart + e, ksplit, int64_t(a.M) * a.N);
    int co = m;
    int64_t pix = n;
    if (a.scatter) {
        const int pi_ = n / a.g.W, pj_ = n - (n / a.g.W) * a.g.W;
        const int ab = m / a.Cout;
        co = m - ab * a.Cout;
        pix = int64_t(2 * pi_ + ab / 2) * a.Wo + 2 * pj_ + ab % 2;
    }
    if (a.bias) v += a.bias[co];
    if (a.act) v = v > 0.f ? v : a.slope * v;
    if (a.act_y && !(bf2f(a.act_y[pix * a.act_ld + a.act_coff + co]) > 0.f)) v *= a.slope;
    a.out[pix * a.out_ld + a.out_coff + co] = f2bf(v);
}


// Weight gradient C[m][n] = sum_p A[p][acoff + m] Bg(p, n) over the pixels
// [p_lo, p_hi) of split z (blockIdx.z): a BM x BN tile per workgroup,
// 64-pixel K slices double-buffered in LDS (one barrier per slice). Both
// operands are pixel-major in memory and channel-major in the matrix-core
// layout, so they are transposed on the way into LDS: a task of 8 channels x
// 4 pixels is four 16-byte loads and eight 8-byte LDS stores. A wave's 64
// tasks are 4 adjacent channel chunks x 16 pixel groups (chunk fastest), so
// a load instruction reads 64 contiguous bytes of each of 16 pixels; the
// 16-byte chunk of an LDS row is XOR-swizzled by bit 4 of the row, which
// keeps the four rows a store instruction writes on distinct banks. Requires M, N, Cb, lda, ld and the
// channel offsets to be multiples of 8 and the split (chunk) a multiple of
// 64. The loads of the next DEPTH slices are in flight while a slice is
// computed (a ring of DEPTH register stages). With one split the sums go
// straight to out, else to partial[z][m][n] for k_wgrad_finish. Bias gradients, per split: the first column of blocks
// sums A over its pixels (bias_from_b = 0: A is the output gradient of a
// convolution), or the first row of blocks sums B (bias_from_b = 1: the
// transposed convolution, whose output gradient is the gathered B).
template <int BM, int BN, int DEPTH>
__global__ __launch_bounds__(256) void k_wgrad_t(const WgradArgs a)
{
    constexpr int BK = 64, LDK = BK + 8;   // LDS rows of 144 B
    constexpr int TA = (BM / 8) * 16, TB = (BN / 8) * 16;
    constexpr int NR = (TA + TB + 255) / 256;
    constexpr int WTM = BM / 32, WTN = BN / 32;
    constexpr int WGM = WTM >= 2 ? 2 : 1, WGN = 4 / WGM;
    constexpr int XM = WTM / WGM, YN = WTN / WGN;
    static_assert(TA % 64 == 0 && WTN % WGN == 0 && XM >= 1 && YN >= 1, "tile shape");
    __shared__ __attribute__((aligned(16))) bf16 As[2][BM * LDK];
    __shared__ __attribute__((aligned(16))) bf16 Bs[2][BN * LDK];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w / WGN, wn = w % WGN;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const Gather &g = a.g;
    const int P = g.H * g.W;
    const int p_lo = blockIdx.z * a.chunk;
    const int p_hi = min(P, p_lo + a.chunk);
    const int nk = p_hi > p_lo ? (p_hi - p_lo + BK - 1) / BK : 0;
    const int pg = (tid >> 2) & 15;   // group of 4 pixels within the slice

    // the task of each round: operand, 8-channel chunk, source offsets
    bool act[NR], isA[NR], val[NR];
    int cc[NR], ty[NR], tx[NR], ch[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int t = tid + 256 * r;
        act[r] = t < TA + TB;
        isA[r] = t < TA;
        {
            const int u = isA[r] ? t : t - TA;   // 4 chunks x 16 pixel groups per wave
            cc[r] = (u & 3) | ((u >> 6) << 2);
        }
        ty[r] = tx[r] = ch[r] = 0;
        if (isA[r]) {
            val[r] = act[r] && m0 + cc[r] * 8 < a.M;
        } else {
            const int nb = n0 + cc[r] * 8;
            val[r] = act[r] && nb < a.N;
            const int tap = val[r] ? nb / g.Cb : 0;
            ch[r] = nb - tap * g.Cb;
            ty[r] = tap / g.tapw;
            tx[r] = tap - ty[r] * g.tapw;
        }
    }
    uint4 rg[DEPTH][NR][4];
    auto load = [&](int kt, int sl) {
        const int p4 = p_lo + kt * BK + pg * 4;
        int i = p4 / g.W, j = p4 - (p4 / g.W) * g.W;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int p = p4 + u;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                rg[sl][r][u] = make_uint4(0, 0, 0, 0);
                if (val[r] && p < p_hi) {
                    if (isA[r]) {
                        rg[sl][r][u] =
                            *reinterpret_cast<const uint4 *>(a.A + int64_t(p) * a.lda + a.acoff + m0 + cc[r] * 8);
                    } else {
                        const int si = i * g.stride + ty[r] + g.d0, sj = j * g.stride + tx[r] + g.d0;
                        if (si >= 0 && si < g.Hs && sj >= 0 && sj < g.Ws)
                            rg[sl][r][u] = *reinterpret_cast<const uint4 *>(g.src + (int64_t(si) * g.Ws + sj) * g.ld +
                                                                            g.coff + ch[r]);
                    }
                }
            }
            if (++j == g.W) {
                j = 0;
                ++i;
            }
        }
    };
    auto store = [&](int sl, int buf) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (!act[r]) continue;
            bf16 *base = isA[r] ? &As[buf][cc[r] * 8 * LDK] : &Bs[buf][cc[r] * 8 * LDK];
            // 16-byte chunk pg/2 of the row, swizzled by bit 4 of the row
            const int col = (((pg >> 1) ^ (((cc[r] >> 1) & 1) << 2)) << 3) + (pg & 1) * 4;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint32_t lo = reinterpret_cast<const uint16_t *>(&rg[sl][r][0])[e] |
                                    (uint32_t(reinterpret_cast<const uint16_t *>(&rg[sl][r][1])[e]) << 16);
                const uint32_t hi = reinterpret_cast<const uint16_t *>(&rg[sl][r][2])[e] |
                                    (uint32_t(reinterpret_cast<const uint16_t *>(&rg[sl][r][3])[e]) << 16);
                *reinterpret_cast<uint2 *>(base + e * LDK + col) = make_uint2(lo, hi);
            }
        }
    };

    const bool bias_a = a.bias_partial != nullptr && !a.bias_from_b && blockIdx.x == 0;
    const bool bias_b = a.bias_partial != nullptr && a.bias_from_b && blockIdx.y == 0;
    float bs[NR][8];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int e = 0; e < 8; ++e) bs[r][e] = 0.f;
    auto bias_add = [&](int sl) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (!(isA[r] ? bias_a : bias_b)) continue;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bf16 *v = reinterpret_cast<const bf16 *>(&rg[sl][r][u]);
#pragma unroll
                for (int e = 0; e < 8; ++e) bs[r][e] += bf2f(v[e]);
            }
        }
    };

    f32x16 acc[XM][YN];
#pragma unroll
    for (int x = 0; x < XM; ++x)
#pragma unroll
        for (int y = 0; y < YN; ++y) acc[x][y] = f32x16{};
    // ring: register stage s holds slice kt with kt % DEPTH == s; slice kt
    // goes to LDS buffer kt & 1 at the end of the previous slice, which frees
    // its stage for slice kt + DEPTH
#pragma unroll
    for (int d = 0; d < DEPTH; ++d)
        if (d < nk) load(d, d);
    if (nk > 0) {
        store(0, 0);
        bias_add(0);
    }
    __syncthreads();
    for (int kt0 = 0; kt0 < nk; kt0 += DEPTH) {
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) {
            const int kt = kt0 + d;
            if (kt < nk) {
                const int buf = kt & 1;
                if (kt + DEPTH < nk) load(kt + DEPTH, d);
#pragma unroll
                for (int kk = 0; kk < BK / 16; ++kk) {
                    bf16x8 av[XM], bv[YN];
                    const int jj = kk * 2 + lane / 32;   // 16-byte chunk of the row
#pragma unroll
                    for (int x = 0; x < XM; ++x) {
                        const int row = (wm * XM + x) * 32 + lane % 32;
                        av[x] = *reinterpret_cast<const bf16x8 *>(
                            &As[buf][row * LDK + ((jj ^ (((row >> 4) & 1) << 2)) << 3)]);
                    }
#pragma unroll
                    for (int y = 0; y < YN; ++y) {
                        const int row = (wn * YN + y) * 32 + lane % 32;
                        bv[y] = *reinterpret_cast<const bf16x8 *>(
                            &Bs[buf][row * LDK + ((jj ^ (((row >> 4) & 1) << 2)) << 3)]);
                    }
#pragma unroll
                    for (int x = 0; x < XM; ++x)
#pragma unroll
                        for (int y = 0; y < YN; ++y)
                            acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[x], bv[y], acc[x][y], 0, 0, 0);
                }
                if (kt + 1 < nk) {
                    store((d + 1) % DEPTH, buf ^ 1);
                    bias_add((d + 1) % DEPTH);
                }
                __syncthreads();
            }
        }
    }
    if (bias_a || bias_b) {
        // the 16 lanes of a channel chunk hold sums over their pixel groups:
        // combine them in a fixed order, then one lane writes the 8 channels
#pragma unroll
        for (int r = 0; r < NR; ++r) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                float v = bs[r][e];
#pragma unroll
                for (int off = 32; off >= 4; off >>= 1) v += __shfl_xor(v, off);
                bs[r][e] = v;
            }
            const bool on = isA[r] ? bias_a : bias_b;
            if (!on || !val[r] || pg != 0) continue;
            const int base = isA[r] ? m0 + cc[r] * 8 : n0 + cc[r] * 8;
            const int len = isA[r] ? a.M : a.N;
            if (isA[r] && a.nsplit == 1) {
#pragma unroll
                for (int e = 0; e < 8; ++e) a.bias_out[base + e] = bs[r][e];
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) a.bias_partial[int64_t(blockIdx.z) * len + base + e] = bs[r][e];
            }
        }
    }
    const bool direct = a.nsplit == 1;
    float *part = a.partial + int64_t(blockIdx.z) * a.M * a.N;
#pragma unroll
    for (int y = 0; y < YN; ++y) {
        const int n = n0 + (wn * YN + y) * 32 + lane % 32;
        if (n >= a.N) continue;
#pragma unroll
        for (int x = 0; x < XM; ++x)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int m = m0 + (wm * XM + x) * 32 + 8 * (i / 4) + 4 * (lane / 32) + (i % 4);
                if (m >= a.M) continue;
                if (direct) a.out[int64_t(m) * a.ldm + int64_t(n) * a.ldn] = acc[x][y][i];
                else part[int64_t(m) * a.N + n] = acc[x][y][i];
            }
    }
}

// Second pass of a split weight gradient: sums the splits of each output in
// order into out[m*ldm + n*ldn]; the threads past M*N sum the bias partials
// ([nsplit][M] from A, or [nsplit][N] from B, where the taps n = tap*Cb + c
// of one channel c are added as well).
__global__ void k_wgrad_finish(const WgradArgs a)
{
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t MN = int64_t(a.M) * a.N;
    if (e < MN) {
        if (a.nsplit == 1) return;   // written by the first pass
        const float s = sum_strided(a.partial + e, a.nsplit, MN);
        const int m = int(e / a.N), n = int(e % a.N);
        a.out[int64_t(m) * a.ldm + int64_t(n) * a.ldn] = s;
        return;
    }
    if (!a.bias_partial) return;
    const int c = int(e - MN);
    if (!a.bias_from_b) {
        if (c < a.M && a.nsplit > 1) a.bias_out[c] = sum_strided(a.bias_partial + c, a.nsplit, a.M);
    } else if (c < a.g.Cb) {
        float t = 0.f;
        for (int tap = 0; tap * a.g.Cb < a.N; ++tap)
            t += sum_strided(a.bias_partial + tap * a.g.Cb + c, a.nsplit, a.N);
        a.bias_out[c] = t;
    }
}

// All deferred second passes of one backward pass in one launch. Entry l of
// tab owns the blocks [bbeg[l], bbeg[l+1]) (its split weight sums, then its
// bias sums), so the entry is the same for the whole block and is looked up
// once. The entry's fin_groups G (1, 2, 4 or 8) splits a block's threads into
// G groups over the splits: thread (g, j) sums the splits z = g, g + G, ...
// of outputs j, j + 256/G, j + 512/G and j + 768/G of the block's 1024/G,
// all four together (eight loads in flight), and the G sums of an output
// are added in LDS in a fixed order.
__global__ __launch_bounds__(256) void k_wgrad_finish_all(const WgradArgs *tab, const int64_t *bbeg, int32_t n)
{
    __shared__ float red[4][256];
    const int64_t blk = blockIdx.x;
    int lo = 0, hi = n;   // the entry holding the block: bbeg[lo] <= blk < bbeg[lo + 1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (bbeg[mid] <= blk) lo = mid;
        else hi = mid;
    }
    const WgradArgs a = tab[lo];
    const int G = a.fin_groups, W = 256 / G;
    const int g = threadIdx.x / W, j = threadIdx.x - g * W;
    const int64_t MN = int64_t(a.M) * a.N;
    const int64_t nw = a.nsplit > 1 ? MN : 0;
    const int64_t nb = a.bias_partial ? (a.bias_from_b ? a.g.Cb : (a.nsplit > 1 ? a.M : 0)) : 0;
    const int64_t k0 = (blk - bbeg[lo]) * (kFinishOutputs / G) + j;
    // weight sums: two accumulators per output over the group's splits
    float s0[4] = {0.f, 0.f, 0.f, 0.f}, s1[4] = {0.f, 0.f, 0.f, 0.f};
    int z = g;
    for (; z + G < a.nsplit; z += 2 * G) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t k = k0 + int64_t(W) * q;
            if (k < nw) {
                s0[q] += a.partial[int64_t(z) * MN + k];
                s1[q] += a.partial[int64_t(z + G) * MN + k];
            }
        }
    }
    if (z < a.nsplit) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t k = k0 + int64_t(W) * q;
            if (k < nw) s0[q] += a.partial[int64_t(z) * MN + k];
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t k = k0 + int64_t(W) * q;
        float t = s0[q] + s1[q];
        if (k >= nw && k < nw + nb) {   // bias sums
            const int c = int(k - nw);
            const int len = a.bias_from_b ? a.N : a.M;
            const int ntap = a.bias_from_b ? a.N / a.g.Cb : 1;
            t = 0.f;
            for (int tap = 0; tap < ntap; ++tap) {
                const float *bp = a.bias_partial + tap * (a.bias_from_b ? a.g.Cb : 0) + c;
                for (int zz = g; zz < a.nsplit; zz += G) t += bp[int64_t(zz) * len];
            }
        }
        red[q][threadIdx.x] = t;
    }
    __syncthreads();
    if (g != 0) return;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t k = k0 + int64_t(W) * q;
        if (k >= nw + nb) continue;
        float v = red[q][j];
        for (int h = 1; h < G; ++h) v += red[q][h * W + j];
        if (k < nw) a.out[(k / a.N) * a.ldm + (k % a.N) * a.ldn] = v;
        else a.bias_out[k - nw] = v;
    }
}

__global__ void k_wgrad_reduce(const float *part, int32_t M, int32_t N, int32_t nsplit, float *out, int32_t ldm,
                               int32_t ldn)
{
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= int64_t(M) * N) return;
    const float s = sum_strided(part + e, nsplit, int64_t(M) * N);
    const int m = int(e / N), n = int(e % N);
    out[int64_t(m) * ldm + int64_t(n) * ldn] = s;
}

// db[c] = sum_p dz[p][coff + c] (C a multiple of 8, at most 2048): each
// thread adds 16-byte chunks (8 channels) of one pixel per row of the block;
// a block covers one pixel split; partial sums per split, reduced in order
// by k_sum_rows.
__global__ __launch_bounds__(256) void k_bias_part(const bf16 *dz, int32_t ld, int32_t coff, int32_t C, int32_t P,
                                                   int32_t chunk, float *part)
{
    __shared__ float red[256][9];
    const int cpp = C / 8;            // 8-channel chunks per pixel
    const int rows = 256 / cpp;       // pixels handled per pass of the block
    const int tid = threadIdx.x;
    const int ch = tid % cpp, pr = tid / cpp;
    const int p0 = blockIdx.x * chunk, p1 = min(P, p0 + chunk);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (pr < rows) {
        for (int p = p0 + pr; p < p1; p += rows) {
            const uint4 v = *reinterpret_cast<const uint4 *>(dz + int64_t(p) * ld + coff + ch * 8);
            const bf16 *b = reinterpret_cast<const bf16 *>(&v);
#pragma unroll
            for (int e = 0; e < 8; ++e) s[e] += bf2f(b[e]);
        }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) red[tid][e] = s[e];
    __syncthreads();
    for (int c = tid; c < C; c += 256) {
        const int cc = c / 8, e = c % 8;
        float t = 0.f;
        for (int r = 0; r < rows; ++r) t += red[r * cpp + cc][e];
        part[int64_t(blockIdx.x) * C + c] = t;
    }
}

// 3x3 convolution of a one-channel image (the input layer), zero padding 1:
// out[p][co] = act(b[co] + sum_t w[co][t] x[p + t]) with bf16 weights and
// inputs and FP32 sums. One thread per pixel and 8 output channels (one
// 16-byte store); the weights are staged in LDS as floats once per block,
// which then strides over the grid.
__global__ __launch_bounds__(256) void k_conv1_fwd(const bf16 *x, int32_t H, int32_t W, const bf16 *w,
                                                   const float *b, int32_t C, int32_t act, float slope, bf16 *out,
                                                   int32_t ld, int32_t coff)
{
    extern __shared__ float wl[];   // [C][9]
    for (int e = threadIdx.x; e < C * 9; e += blockDim.x) wl[e] = bf2f(w[e]);
    __syncthreads();
    const int cpp = C / 8;
    const int64_t n = int64_t(H) * W * cpp;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += stride) {
        const int c8 = int(t % cpp);
        const int p = int(t / cpp);
        const int i = p / W, j = p - (p / W) * W;
        float xv[9];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int si = i + tap / 3 - 1, sj = j + tap % 3 - 1;
            xv[tap] = (si >= 0 && si < H && sj >= 0 && sj < W) ? bf2f(x[si * W + sj]) : 0.f;
        }
        bf16 o[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int co = c8 * 8 + e;
            float acc = 0.f;
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) acc = __builtin_fmaf(wl[co * 9 + tap], xv[tap], acc);
            float v = acc + b[co];
            if (act) v = v > 0.f ? v : slope * v;
            o[e] = f2bf(v);
        }
        *reinterpret_cast<uint4 *>(out + int64_t(p) * ld + coff + c8 * 8) = *reinterpret_cast<const uint4 *>(o);
    }
}

// Weight and bias gradients of the input layer: dW[co][t] = sum_p dz[p][co]
// x[p + t] and db[co] = sum_p dz[p][co]. Block (s, c8) sums pixel split s for
// channels 8 c8 .. 8 c8 + 7: per-thread sums over a strided pixel subset,
// then a wave-shuffle and LDS reduction in a fixed order; partial[s][C][10]
// (9 taps, then the bias).
__global__ __launch_bounds__(256) void k_conv1_wgrad(const bf16 *dz, int32_t ld, int32_t zoff, const bf16 *x,
                                                     int32_t H, int32_t W, int32_t C, int32_t chunk, float *part)
{
    __shared__ float red[4][80];
    const int c8 = blockIdx.y, sp = blockIdx.x;
    const int P = H * W;
    const int p0 = sp * chunk, p1 = min(P, p0 + chunk);
    float acc[8][10];
#pragma unroll
    for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int k = 0; k < 10; ++k) acc[e][k] = 0.f;
#pragma unroll 4
    for (int p = p0 + int(threadIdx.x); p < p1; p += blockDim.x) {
        const uint4 v = *reinterpret_cast<const uint4 *>(dz + int64_t(p) * ld + zoff + c8 * 8);
        const bf16 *d = reinterpret_cast<const bf16 *>(&v);
        const int i = p / W, j = p - (p / W) * W;
        float xv[9];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int si = i + tap / 3 - 1, sj = j + tap % 3 - 1;
            xv[tap] = (si >= 0 && si < H && sj >= 0 && sj < W) ? bf2f(x[si * W + sj]) : 0.f;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float de = bf2f(d[e]);
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) acc[e][tap] = __builtin_fmaf(de, xv[tap], acc[e][tap]);
            acc[e][9] += de;
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            float v = acc[e][k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0) red[wv][e * 10 + k] = v;
        }
    __syncthreads();
    if (threadIdx.x < 80) {
        const float v = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
        part[(int64_t(sp) * C + c8 * 8) * 10 + threadIdx.x] = v;
    }
}

// sums partial[s][C][10] over the splits in order and scatters into dW[C][9]
// and db[C]
__global__ void k_conv1_wgrad_finish(const float *part, int32_t nsplit, int32_t C, float *dw, float *db)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= C * 10) return;
    const float v = sum_strided(part + e, nsplit, int64_t(C) * 10);
    const int co = e / 10, k = e - (e / 10) * 10;
    if (k < 9) dw[co * 9 + k] = v;
    else db[co] = v;
}

__global__ void k_sum_rows(const float *part, int32_t rows, int32_t C, float *out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    out[c] = sum_strided(part + c, rows, C);
}

__global__ void k_act_bwd(bf16 *dz, int32_t ldz, int32_t zoff, const bf16 *dy, int32_t ldy, int32_t yoff,
                          const bf16 *y, int32_t ld, int32_t coff, int32_t C, int32_t P, float slope)
{
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= int64_t(P) * C) return;
    const int64_t p = e / C;
    const int c = int(e - p * C);
    const float d = bf2f(dy[p * ldy + yoff + c]);
    const float yy = bf2f(y[p * ld + coff + c]);
    dz[p * ldz + zoff + c] = f2bf(yy > 0.f ? d : slope * d);
}

__global__ void k_pool_fwd(const bf16 *in, int32_t ldi, int32_t coff, int32_t C, int32_t H, int32_t W, bf16 *out)
{
    const int Ho = H / 2, Wo = W / 2;
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= int64_t(Ho) * Wo * C) return;
    const int c = int(e % C);
    const int64_t q = e / C;
    const int i = int(q / Wo), j = int(q % Wo);
    float s = 0.f;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const int y = 2 * i + dy, x = 2 * j + dx;
            if (y >= 0 && y < H && x >= 0 && x < W) s += bf2f(in[(int64_t(y) * W + x) * ldi + coff + c]);
        }
    out[q * C + c] = f2bf(s * (1.0f / 9.0f));
}

__global__ void k_pool_bwd(const bf16 *dout, int32_t C, int32_t H, int32_t W, bf16 *din, int32_t ldi, int32_t coff,
                           int32_t accumulate, const bf16 *act_y, float slope)
{
    const int Ho = H / 2, Wo = W / 2;
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= int64_t(H) * W * C) return;
    const int c = int(e % C);
    const int64_t q = e / C;
    const int y = int(q / W), x = int(q % W);
    float s = 0.f;
    for (int i = (y - 1 + 1) / 2; i <= (y + 1) / 2; ++i) {
        if (i < 0 || i >= Ho || 2 * i - y > 1 || y - 2 * i > 1) continue;
        for (int j = (x - 1 + 1) / 2; j <= (x + 1) / 2; ++j) {
            if (j < 0 || j >= Wo || 2 * j - x > 1 || x - 2 * j > 1) continue;
            s += bf2f(dout[(int64_t(i) * Wo + j) * C + c]);
        }
    }
    s *= (1.0f / 9.0f);
    bf16 *dst = din + q * ldi + coff + c;
    if (accumulate) s += bf2f(*dst);
    if (act_y && !(bf2f(act_y[q * ldi + coff + c]) > 0.f)) s *= slope;
    *dst = f2bf(s);
}

// Vectorised pooling (C, ldi and coff multiples of 8): one thread per pixel
// and 8 channels, 16-byte loads and stores; same sums in the same order as
// the scalar kernels.
__global__ void k_pool_fwd8(const bf16 *in, int32_t ldi, int32_t coff, int32_t C, int32_t H, int32_t W, bf16 *out)
{
    const int Ho = H / 2, Wo = W / 2, C8 = C / 8;
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= int64_t(Ho) * Wo * C8) return;
    const int c8 = int(e % C8);
    const int64_t q = e / C8;
    const int i = int(q / Wo), j = int(q % Wo);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const int y = 2 * i + dy, x = 2 * j + dx;
            if (y < 0 || y >= H || x < 0 || x >= W) continue;
            const uint4 v = *reinterpret_cast<const uint4 *>(in + (int64_t(y) * W + x) * ldi + coff + c8 * 8);
            const bf16 *b = reinterpret_cast<const bf16 *>(&v);
#pragma unroll
            for (int k = 0; k < 8; ++k) s[k] += bf2f(b[k]);
        }
    bf16 o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = f2bf(s[k] * (1.0f / 9.0f));
    *reinterpret_cast<uint4 *>(out + q * C + c8 * 8) = *reinterpret_cast<const uint4 *>(o);
}

__global__ void k_pool_bwd8(const bf16 *dout, int32_t C, int32_t H, int32_t W, bf16 *din, int32_t ldi, int32_t coff,
                            int32_t accumulate, const bf16 *act_y, float slope)
{
    const int Ho = H / 2, Wo = W / 2, C8 = C / 8;
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= int64_t(H) * W * C8) return;
    const int c8 = int(e % C8);
    const int64_t q = e / C8;
    const int y = int(q / W), x = int(q % W);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int i = (y - 1 + 1) / 2; i <= (y + 1) / 2; ++i) {
        if (i < 0 || i >= Ho || 2 * i - y > 1 || y - 2 * i > 1) continue;
        for (int j = (x - 1 + 1) / 2; j <= (x + 1) / 2; ++j) {
            if (j < 0 || j >= Wo || 2 * j - x > 1 || x - 2 * j > 1) continue;
            const uint4 v = *reinterpret_cast<const uint4 *>(dout + (int64_t(i) * Wo + j) * C + c8 * 8);
            const bf16 *b = reinterpret_cast<const bf16 *>(&v);
#pragma unroll
            for (int k = 0; k < 8; ++k) s[k] += bf2f(b[k]);
        }
    }
    bf16 *dst = din + q * ldi + coff + c8 * 8;
    float prev[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (accumulate) {
        const uint4 v = *reinterpret_cast<const uint4 *>(dst);
        const bf16 *b = reinterpret_cast<const bf16 *>(&v);
#pragma unroll
        for (int k = 0; k < 8; ++k) prev[k] = bf2f(b[k]);
    }
    float yy[8] = {1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f};
    if (act_y) {
        const uint4 v = *reinterpret_cast<const uint4 *>(act_y + q * ldi + coff + c8 * 8);
        const bf16 *b = reinterpret_cast<const bf16 *>(&v);
#pragma unroll
        for (int k = 0; k < 8; ++k) yy[k] = bf2f(b[k]);
    }
    bf16 o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        float v = s[k] * (1.0f / 9.0f);
        if (accumulate) v += prev[k];
        if (act_y && !(yy[k] > 0.f)) v *= slope;
        o[k] = f2bf(v);
    }
    *reinterpret_cast<uint4 *>(dst) = *reinterpret_cast<const uint4 *>(o);
}

// Backward of the 1x1 output convolution for C a multiple of 8 with C/8 <=
// 256: a block of 256 pixels; thread t takes the 8-channel chunk t % (C/8)
// of every (256 / (C/8))-th pixel, writes dx = w dy (times the activation
// derivative at x) with 16-byte stores and sums dy x per channel; the sums
// of the block are combined in LDS in a fixed order into part_w[block][C]
// and the sum of dy into part_w[block][C].
__global__ __launch_bounds__(256) void k_outc_bwd8(const bf16 *x, int32_t C, int32_t P, const float *w,
                                                   const float *dy, bf16 *dx, float *part_w, float slope)
{
    __shared__ float red[2048 + 256];
    const int C8 = C / 8, rows = 256 / C8;
    const int tid = threadIdx.x, cc = tid % C8, ps = tid / C8;
    const int p0 = blockIdx.x * 256;
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, sd = 0.f;
    float wc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) wc[k] = w[cc * 8 + k];
    if (ps < rows) {
        for (int p = p0 + ps; p < min(P, p0 + 256); p += rows) {
            const float d = dy[p];
            const uint4 v = *reinterpret_cast<const uint4 *>(x + int64_t(p) * C + cc * 8);
            const bf16 *xb = reinterpret_cast<const bf16 *>(&v);
            bf16 o[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const float xv = bf2f(xb[k]);
                const float gx = wc[k] * d;
                o[k] = f2bf(xv > 0.f ? gx : slope * gx);
                s[k] += d * xv;
            }
            sd += d;
            *reinterpret_cast<uint4 *>(dx + int64_t(p) * C + cc * 8) = *reinterpret_cast<const uint4 *>(o);
        }
        // rows x C channel sums, then rows sums of dy
#pragma unroll
        for (int k = 0; k < 8; ++k) red[ps * C + cc * 8 + k] = s[k];
        if (cc == 0) red[2048 + ps] = sd;
    }
    __syncthreads();
    for (int c = tid; c <= C; c += 256) {
        float t = 0.f;
        if (c < C)
            for (int r = 0; r < rows; ++r) t += red[r * C + c];
        else
            for (int r = 0; r < rows; ++r) t += red[2048 + r];
        part_w[int64_t(blockIdx.x) * (C + 1) + c] = t;
    }
}

// max |x| in two passes: per-block maxima, then the maximum of those (the
// result does not depend on the order)
__global__ __launch_bounds__(256) void k_absmax_part(const float *x, int64_t n, float *part)
{
    __shared__ float red[256];
    float m = 0.f;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) m = fmaxf(m, fabsf(x[i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + k]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// 1x1 output convolution with 16-byte loads (C a multiple of 8): the same
// sum over the channels in the same order as k_outc_fwd
__global__ __launch_bounds__(256) void k_outc_fwd8(const bf16 *x, int32_t C, int32_t P, const float *w, const float *b,
                                                   float *y)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    float s = b[0];
    for (int c = 0; c < C; c += 8) {
        const uint4 v = *reinterpret_cast<const uint4 *>(x + int64_t(p) * C + c);
        const bf16 *xb = reinterpret_cast<const bf16 *>(&v);
#pragma unroll
        for (int k = 0; k < 8; ++k) s += w[c + k] * bf2f(xb[k]);
    }
    y[p] = s;
}

__global__ void k_outc_fwd(const bf16 *x, int32_t C, int32_t P, const float *w, const float *b, float *y)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    float s = b[0];
    for (int c = 0; c < C; ++c) s += w[c] * bf2f(x[int64_t(p) * C + c]);
    y[p] = s;
}

__global__ __launch_bounds__(256) void k_mse(const float *y, const float *t, int32_t P, double *partials, float *dy)
{
    __shared__ double red[256];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (p < P) {
        const float d = y[p] - t[p];
        s = double(d) * double(d);
        dy[p] = 2.0f * d / float(P);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_outc_bwd(const bf16 *x, int32_t C, int32_t P, const float *w,
                                                  const float *dy, bf16 *dx, float *part_w, float slope)
{
    // block of 256 pixels; part_w[block][c] for c < C, part_w[block][C] = sum dy
    __shared__ float red[256];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const float d = p < P ? dy[p] : 0.f;
    for (int c = 0; c <= C; ++c) {
        float v = 0.f;
        if (p < P) {
            if (c < C) {
                const float xv = bf2f(x[int64_t(p) * C + c]);
                const float gx = w[c] * d;
                dx[int64_t(p) * C + c] = f2bf(xv > 0.f ? gx : slope * gx);
                v = d * xv;
            } else {
                v = d;
            }
        }
        red[threadIdx.x] = v;
        __syncthreads();
        for (int k = 128; k > 0; k >>= 1) {
            if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
            __syncthreads();
        }
        if (threadIdx.x == 0) part_w[int64_t(blockIdx.x) * (C + 1) + c] = red[0];
        __syncthreads();
    }
}

// dw[c], db: block c reduces column c of the [nblk][C+1] partials with 256
// threads (fixed order)
__global__ __launch_bounds__(256) void k_outc_reduce(const float *part, int32_t C, int32_t nblk, float *dw, float *db)
{
    __shared__ float red[256];
    const int c = blockIdx.x;
    float s = 0.f;
    for (int b = threadIdx.x; b < nblk; b += 256) s += part[int64_t(b) * (C + 1) + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (c < C) dw[c] = red[0];
        else db[0] = red[0];
    }
}

__global__ __launch_bounds__(256) void k_sum_d(const double *p, int32_t n, double *out, float scale, float *out_f)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += p[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (out) *out = red[0] * scale;
        if (out_f) *out_f = float(red[0] * scale);
    }
}

__global__ void k_adam(float *p, const float *g, float *m, float *v, bf16 *pb, int64_t n, const float *hyper,
                       float beta1, float beta2, float eps)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float lr = hyper[0], c1 = hyper[1], c2 = hyper[2];
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float upd = (mi / c1) / (sqrtf(vi / c2) + eps);
    const float pi = p[i] - lr * upd;
    p[i] = pi;
    pb[i] = f2bf(pi);
}

// The bf16 data-gradient matrices from the bf16 weights, a transpose through
// LDS in 64 x 64 tiles with 16-byte loads and stores (coalesced on both
// sides). Weight tensor s is an R x C matrix at pb + off: a 3x3 convolution
// [co][tap*Cin + ci] (R = Cout, C = 9 Cin) going to aux[ci][(8 - tap)*Cout +
// co]; a 2x2 transposed convolution [ab*Cout + co][ci] (R = 4 Cout, C = Cin)
// going to aux[ci][ab*Cout + co]. R, C, off and aux_off are multiples of 8.
// Block t is tile t - tile0[s] of tensor s (row-major over the tiles).
__global__ __launch_bounds__(256) void k_aux_from_pb(const AuxSeg *segs, int32_t nseg, const bf16 *pb, bf16 *aux)
{
    __shared__ uint16_t tl[64][66];
    const int64_t t = blockIdx.x;
    int lo = 0, hi = nseg;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (segs[mid].tile0 <= t) lo = mid;
        else hi = mid;
    }
    const AuxSeg sg = segs[lo];
    const int R = sg.kind == 0 ? sg.cout : 4 * sg.cout;
    const int C = sg.kind == 0 ? 9 * sg.cin : sg.cin;
    const int tc = (C + 63) / 64;
    const int64_t local = t - sg.tile0;
    const int r0 = int(local / tc) * 64, c0 = int(local % tc) * 64;
    const int tid = threadIdx.x;
    // load: 64 rows x 8 chunks of 8 columns
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int e = tid + 256 * i, r = e >> 3, ch = (e & 7) * 8;
        if (r0 + r < R && c0 + ch < C) {
            const uint4 v = *reinterpret_cast<const uint4 *>(pb + sg.off + int64_t(r0 + r) * C + c0 + ch);
            const uint16_t *h = reinterpret_cast<const uint16_t *>(&v);
#pragma unroll
            for (int k = 0; k < 8; ++k) tl[r][ch + k] = h[k];
        }
    }
    __syncthreads();
    // store: 64 columns x 8 chunks of 8 rows
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int e = tid + 256 * i, c = e >> 3, rh = (e & 7) * 8;
        if (r0 + rh >= R || c0 + c >= C) continue;
        const int cc = c0 + c;
        int64_t dst;
        if (sg.kind == 0) {
            const int tap = cc / sg.cin, ci = cc - tap * sg.cin;
            dst = int64_t(ci) * 9 * sg.cout + int64_t(8 - tap) * sg.cout + r0 + rh;
        } else {
            dst = int64_t(cc) * R + r0 + rh;
        }
        uint16_t h[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) h[k] = tl[rh + k][c];
        *reinterpret_cast<uint4 *>(aux + sg.aux_off + dst) = *reinterpret_cast<const uint4 *>(h);
    }
}

__global__ void k_to_bf16(const float *x, bf16 *y, int64_t n)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

__global__ __launch_bounds__(256) void k_absmax(const float *x, int64_t n, float *out)
{
    __shared__ float red[256];
    float m = 0.f;
    for (int64_t i = threadIdx.x; i < n; i += 256) m = fmaxf(m, fabsf(x[i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + k]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

__device__ __forceinline__ int reflect(int k, int n)
{
    if (n == 1) return 0;
    while (k < 0 || k >= n) {
        if (k < 0) k = -k;
        if (k >= n) k = 2 * (n - 1) - k;
    }
    return k;
}

__global__ void k_pad_norm(const float *src, int32_t nz, int32_t nx, int32_t H, int32_t W, int32_t py, int32_t px,
                           const float *maxabs, bf16 *dst_b, float *dst_f)
{
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= int64_t(H) * W) return;
    const int i = int(e / W), j = int(e % W);
    const float mx = maxabs[0];
    const float s = mx > 0.f ? 1.0f / mx : 0.f;
    const float v = src[int64_t(reflect(i - py, nz)) * nx + reflect(j - px, nx)] * s;
    if (dst_b) dst_b[e] = f2bf(v);
    if (dst_f) dst_f[e] = v;
}

__global__ void k_crop_scale(const float *y, int32_t H, int32_t W, int32_t py, int32_t px, int32_t nz, int32_t nx,
                             const float *maxabs, float *out)
{
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= int64_t(nz) * nx) return;
    const int i = int(e / nx), j = int(e % nx);
    (void)H;
    out[e] = y[int64_t(i + py) * W + j + px] * maxabs[0];
}

__global__ void k_fill_f(float *p, int64_t n, float v)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

inline unsigned nblocks(int64_t n, int b = 256) { return unsigned((n + b - 1) / b); }

}  // namespace

hipError_t conv1_fwd(const bf16 *x, int32_t H, int32_t W, const bf16 *w, const float *b, int32_t C, int32_t act,
                     float slope, bf16 *out, int32_t ld, int32_t coff, hipStream_t s)
{
    if (C % 8 || C > 1024 || ld % 8 || coff % 8) return hipErrorInvalidValue;   // weights: <= 36 KB of LDS
    const int64_t threads = int64_t(H) * W * (C / 8);
    if (threads == 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((threads + 255) / 256, 2048);
    hipLaunchKernelGGL(k_conv1_fwd, dim3(unsigned(blocks)), dim3(256), size_t(C) * 9 * sizeof(float), s, x, H, W, w,
                       b, C, act, slope, out, ld, coff);
    return hipGetLastError();
}

hipError_t conv1_wgrad(const bf16 *dz, int32_t ld, int32_t zoff, const bf16 *x, int32_t H, int32_t W, int32_t C,
                       float *part, int64_t part_floats, float *dw, float *db, hipStream_t s)
{
    if (C % 8 || C > 2048 || ld % 8 || zoff % 8) return hipErrorInvalidValue;
    const int P = H * W;
    if (P == 0) return hipSuccess;
    int nsplit = std::max(1, std::min((P + 2047) / 2048, 512));
    nsplit = int(std::min<int64_t>(nsplit, part_floats / (int64_t(C) * 10)));
    if (nsplit < 1) return hipErrorInvalidValue;
    const int chunk = (P + nsplit - 1) / nsplit;
    hipLaunchKernelGGL(k_conv1_wgrad, dim3(nsplit, C / 8), dim3(256), 0, s, dz, ld, zoff, x, H, W, C, chunk, part);
    hipLaunchKernelGGL(k_conv1_wgrad_finish, dim3(nblocks(C * 10)), dim3(256), 0, s, part, nsplit, C, dw, db);
    return hipGetLastError();
}

hipError_t gemm(const GemmArgs &a_in, hipStream_t s)
{
    if (a_in.M <= 0 || a_in.N <= 0) return hipSuccess;
    GemmArgs a = a_in;
    // 8-byte epilogue stores of 4 consecutive channels (and 16-byte split-K
    // partials) when every channel offset and stride allows them
    a.out_vec = a.M % 4 == 0 && a.out_ld % 4 == 0 && a.out_coff % 4 == 0 && (!a.scatter || a.Cout % 4 == 0) &&
                (!a.act_y || (a.act_ld % 4 == 0 && a.act_coff % 4 == 0));
    const bool vec = a.K % kBK == 0 && a.g.Cb % 8 == 0 && a.lda % 8 == 0 && a.g.ld % 8 == 0 && a.g.coff % 8 == 0;
    // thin outputs use 32 x 256 tiles, wide ones 64 x 128; small problems
    // (the coarse levels) keep 64 x 64 tiles so that enough blocks run
    const int64_t blocks_wide = int64_t(nblocks(a.N, 128)) * nblocks(a.M, 64);
    const int64_t blocks_big = int64_t(nblocks(a.N, 128)) * nblocks(a.M, 128);
    if (vec && a.K % 64 == 0 && a.M >= 128 && blocks_big >= 240) {
        hipLaunchKernelGGL(k_gemm2, dim3(nblocks(a.N, 128), nblocks(a.M, 128)), dim3(256), 0, s, a);
    } else if (vec && a.K % 64 == 0 && a.M >= 128 && a.kpart && a.K >= 1024) {
        // few output tiles and a long K: split K over up to ~480 workgroups
        // (at least 4 slices each), then sum the parts in order
        int ks = int(std::min<int64_t>(480 / blocks_big, a.K / 256));
        ks = int(std::min<int64_t>(ks, a.kpart_cap / (int64_t(a.M) * a.N)));
        ks = std::max(ks, 1);
        hipLaunchKernelGGL(k_gemm2, dim3(nblocks(a.N, 128), nblocks(a.M, 128), unsigned(ks)), dim3(256), 0, s, a);
        if (ks > 1) {
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_gemm_finish, dim3(nblocks(int64_t(a.M) * a.N)), dim3(256), 0, s, a, ks);
        }
    } else if (a.M <= 32) {
        const dim3 grid(nblocks(a.N, 256), nblocks(a.M, 32));
        if (vec) hipLaunchKernelGGL((k_gemm_v<1, 4, 2, 4>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_gemm<1, 4, 2, false>), grid, dim3(256), 0, s, a);
    } else if (blocks_wide >= 512) {
        const dim3 grid(nblocks(a.N, 128), nblocks(a.M, 64));
        if (vec) hipLaunchKernelGGL((k_gemm_v<2, 2, 2, 4>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_gemm<2, 2, 2, false>), grid, dim3(256), 0, s, a);
    } else {
        const dim3 grid(nblocks(a.N, 64), nblocks(a.M, 64));
        if (vec) hipLaunchKernelGGL((k_gemm_v<2, 2, 1, 4>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_gemm<2, 2, 1, false>), grid, dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

bool wgrad_vec(const WgradArgs &a)
{
    return a.g.Cb % 8 == 0 && a.lda % 8 == 0 && a.acoff % 8 == 0 && a.g.ld % 8 == 0 && a.g.coff % 8 == 0 &&
           a.M % 8 == 0 && a.N % 8 == 0 && a.chunk % 64 == 0;
}

int wgrad_finish_groups(const WgradArgs &a)
{
    return a.nsplit >= 64 ? 8 : a.nsplit >= 32 ? 4 : a.nsplit >= 16 ? 2 : 1;
}

int64_t wgrad_finish_count(const WgradArgs &a)
{
    if (a.M <= 0 || a.N <= 0 || !wgrad_vec(a)) return 0;
    const int64_t nw = a.nsplit > 1 ? int64_t(a.M) * a.N : 0;
    const int64_t nb = !a.bias_partial ? 0 : (a.bias_from_b ? a.g.Cb : (a.nsplit > 1 ? a.M : 0));
    return nw + nb;
}

hipError_t wgrad_finish_all(const WgradArgs *tab, const int64_t *bbeg, int32_t n, int64_t nblk, hipStream_t s)
{
    if (n <= 0 || nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_wgrad_finish_all, dim3(unsigned(nblk)), dim3(256), 0, s, tab, bbeg, n);
    return hipGetLastError();
}

hipError_t wgrad(const WgradArgs &a, hipStream_t s, bool defer_finish)
{
    if (a.M <= 0 || a.N <= 0) return hipSuccess;
    if (a.nsplit < 1) return hipErrorInvalidValue;
    const bool vec = wgrad_vec(a);
    if (!vec) {
        // generic path (unaligned channels): partials, then the ordered sums
        if (a.bias_from_b) return hipErrorInvalidValue;
        const dim3 grid(nblocks(a.N, 64), nblocks(a.M, 64), unsigned(a.nsplit));
        hipLaunchKernelGGL(k_wgrad<false>, grid, dim3(256), 0, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_wgrad_reduce, dim3(nblocks(int64_t(a.M) * a.N)), dim3(256), 0, s, a.partial, a.M, a.N,
                           a.nsplit, a.out, a.ldm, a.ldn);
        e = hipGetLastError();
        if (e != hipSuccess || !a.bias_partial) return e;
        hipLaunchKernelGGL(k_sum_rows, dim3(nblocks(a.M)), dim3(256), 0, s, a.bias_partial, a.nsplit, a.M,
                           a.bias_out);
        return hipGetLastError();
    }
    const dim3 grid(nblocks(a.N, a.bn), nblocks(a.M, a.bm), unsigned(a.nsplit));
    if (a.bm == 128 && a.bn == 128) hipLaunchKernelGGL((k_wgrad_t<128, 128, 3>), grid, dim3(256), 0, s, a);
    else if (a.bm == 64 && a.bn == 128) hipLaunchKernelGGL((k_wgrad_t<64, 128, 3>), grid, dim3(256), 0, s, a);
    else if (a.bm == 32 && a.bn == 128) hipLaunchKernelGGL((k_wgrad_t<32, 128, 3>), grid, dim3(256), 0, s, a);
    else if (a.bm == 64 && a.bn == 64) hipLaunchKernelGGL((k_wgrad_t<64, 64, 3>), grid, dim3(256), 0, s, a);
    else return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // one split and a bias from A: the first pass wrote everything
    if ((a.nsplit == 1 && !a.bias_from_b) || defer_finish) return hipSuccess;
    const int64_t nbias = a.bias_partial ? (a.bias_from_b ? a.g.Cb : a.M) : 0;
    hipLaunchKernelGGL(k_wgrad_finish, dim3(nblocks(int64_t(a.M) * a.N + nbias)), dim3(256), 0, s, a);
    return hipGetLastError();
}


hipError_t bias_grad(const bf16 *dz, int32_t ld, int32_t coff, int32_t C, int32_t P, float *db, float *scratch,
                     int32_t nsplit, hipStream_t s);

hipError_t act_bwd(bf16 *dz, int32_t ldz, int32_t zoff, const bf16 *dy, int32_t ldy, int32_t yoff, const bf16 *y,
                   int32_t ld, int32_t coff, int32_t C, int32_t P, float slope, hipStream_t s)
{
    hipLaunchKernelGGL(k_act_bwd, dim3(nblocks(int64_t(P) * C)), dim3(256), 0, s, dz, ldz, zoff, dy, ldy, yoff, y, ld,
                       coff, C, P, slope);
    return hipGetLastError();
}

hipError_t pool_fwd(const bf16 *in, int32_t ldi, int32_t coff, int32_t C, int32_t H, int32_t W, bf16 *out,
                    hipStream_t s)
{
    if (C % 8 == 0 && ldi % 8 == 0 && coff % 8 == 0) {
        hipLaunchKernelGGL(k_pool_fwd8, dim3(nblocks(int64_t(H / 2) * (W / 2) * (C / 8))), dim3(256), 0, s, in, ldi,
                           coff, C, H, W, out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_pool_fwd, dim3(nblocks(int64_t(H / 2) * (W / 2) * C)), dim3(256), 0, s, in, ldi, coff, C, H,
                       W, out);
    return hipGetLastError();
}

hipError_t pool_bwd(const bf16 *dout, int32_t C, int32_t H, int32_t W, bf16 *din, int32_t ldi, int32_t coff,
                    int32_t accumulate, const bf16 *act_y, float slope, hipStream_t s)
{
    if (C % 8 == 0 && ldi % 8 == 0 && coff % 8 == 0) {
        hipLaunchKernelGGL(k_pool_bwd8, dim3(nblocks(int64_t(H) * W * (C / 8))), dim3(256), 0, s, dout, C, H, W, din,
                           ldi, coff, accumulate, act_y, slope);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_pool_bwd, dim3(nblocks(int64_t(H) * W * C)), dim3(256), 0, s, dout, C, H, W, din, ldi, coff,
                       accumulate, act_y, slope);
    return hipGetLastError();
}

hipError_t outc_fwd(const bf16 *x, int32_t C, int32_t P, const float *w, const float *b, float *y, hipStream_t s)
{
    if (C % 8 == 0) {
        hipLaunchKernelGGL(k_outc_fwd8, dim3(nblocks(P)), dim3(256), 0, s, x, C, P, w, b, y);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_outc_fwd, dim3(nblocks(P)), dim3(256), 0, s, x, C, P, w, b, y);
    return hipGetLastError();
}

hipError_t mse(const float *y, const float *t, int32_t P, double *partials, int32_t nblk, float *dy, hipStream_t s)
{
    (void)nblk;
    hipLaunchKernelGGL(k_mse, dim3(nblocks(P)), dim3(256), 0, s, y, t, P, partials, dy);
    return hipGetLastError();
}

hipError_t outc_bwd(const bf16 *x, int32_t C, int32_t P, const float *w, const float *dy, bf16 *dx, float *part_w,
                    int32_t nblk, float slope, hipStream_t s)
{
    (void)nblk;
    if (C % 8 == 0 && C <= 2048) {
        hipLaunchKernelGGL(k_outc_bwd8, dim3(nblocks(P)), dim3(256), 0, s, x, C, P, w, dy, dx, part_w, slope);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_outc_bwd, dim3(nblocks(P)), dim3(256), 0, s, x, C, P, w, dy, dx, part_w, slope);
    return hipGetLastError();
}

hipError_t outc_wgrad_reduce(const float *part_w, int32_t C, int32_t nblk, float *dw, float *db, hipStream_t s)
{
    hipLaunchKernelGGL(k_outc_reduce, dim3(unsigned(C + 1)), dim3(256), 0, s, part_w, C, nblk, dw, db);
    return hipGetLastError();
}

hipError_t sum_partials_d(const double *p, int32_t n, double *out, float scale, float *out_f, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_d, dim3(1), dim3(256), 0, s, p, n, out, scale, out_f);
    return hipGetLastError();
}

hipError_t adam(float *p, const float *g, float *m, float *v, bf16 *pb, int64_t n, const float *hyper, float beta1,
                float beta2, float eps, hipStream_t s)
{
    hipLaunchKernelGGL(k_adam, dim3(nblocks(n)), dim3(256), 0, s, p, g, m, v, pb, n, hyper, beta1, beta2, eps);
    return hipGetLastError();
}

hipError_t aux_from_pb(const AuxSeg *segs, int32_t nseg, int64_t ntiles, const bf16 *pb, bf16 *aux, hipStream_t s)
{
    if (nseg <= 0 || ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_aux_from_pb, dim3(unsigned(ntiles)), dim3(256), 0, s, segs, nseg, pb, aux);
    return hipGetLastError();
}

hipError_t to_bf16(const float *x, bf16 *y, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_bf16, dim3(nblocks(n)), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}

hipError_t absmax(const float *x, int64_t n, float *out, float *part, hipStream_t s)
{
    hipLaunchKernelGGL(k_absmax_part, dim3(kAbsmaxBlocks), dim3(256), 0, s, x, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_absmax, dim3(1), dim3(256), 0, s, part, int64_t(kAbsmaxBlocks), out);
    return hipGetLastError();
}

hipError_t pad_norm(const float *src, int32_t nz, int32_t nx, int32_t H, int32_t W, int32_t py, int32_t px,
                    const float *maxabs, bf16 *dst_b, float *dst_f, hipStream_t s)
{
    hipLaunchKernelGGL(k_pad_norm, dim3(nblocks(int64_t(H) * W)), dim3(256), 0, s, src, nz, nx, H, W, py, px, maxabs,
                       dst_b, dst_f);
    return hipGetLastError();
}

hipError_t crop_scale(const float *y, int32_t H, int32_t W, int32_t py, int32_t px, int32_t nz, int32_t nx,
                      const float *maxabs, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_crop_scale, dim3(nblocks(int64_t(nz) * nx)), dim3(256), 0, s, y, H, W, py, px, nz, nx,
                       maxabs, out);
    return hipGetLastError();
}

hipError_t fill_f(float *p, int64_t n, float v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f, dim3(nblocks(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t bias_grad(const bf16 *dz, int32_t ld, int32_t coff, int32_t C, int32_t P, float *db, float *scratch,
                     int32_t nsplit, hipStream_t s)
{
    if (C % 8 || C > 2048 || ld % 8 || coff % 8) return hipErrorInvalidValue;
    const int chunk = (P + nsplit - 1) / nsplit;
    hipLaunchKernelGGL(k_bias_part, dim3(unsigned(nsplit)), dim3(256), 0, s, dz, ld, coff, C, P, chunk, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_rows, dim3(nblocks(C)), dim3(256), 0, s, scratch, nsplit, C, db);
    return hipGetLastError();
}

}  // namespace dbl
