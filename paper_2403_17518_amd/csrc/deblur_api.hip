// Deblurring network runtime and C ABI (include/deblur.h): parameter layout,
// activation buffers, the forward and backward layer schedules, Adam with a
// cosine learning-rate schedule, input scaling/padding, save/load.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/deblur.h"
#include "deblur_internal.h"
#include "internal.h"

using namespace dbl;

namespace {

constexpr float kBeta1 = 0.9f, kBeta2 = 0.999f, kEps = 1e-8f;
constexpr uint32_t kMagic = 0x44424c31;  // "DBL1"

struct ConvL {
    int cin, cout;
    int64_t w, b;      // offsets into the flat parameter vector
    int64_t aux;       // offset of the data-gradient weights (bf16)
    char name[24];     // layer name in timing records
};

// one timed GEMM launch (per-layer profiling)
struct ProfRec {
    const char *name;
    int pass, M, N, K;
    hipEvent_t e0, e1;
};

enum Kind { KW3 = 0, KB = 1, KWT = 2, KW1 = 3 };
struct Entry {
    int kind, cin, cout;
    int64_t off, n;
};

struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct deblur_net {
    deblur_cfg cfg{};
    int device = 0;
    std::string err;
    int D = 0;
    std::vector<int> C, H, W, P;
    ConvL inc[2];
    std::vector<ConvL> down1, down2, upT, up1, up2;  // index by level
    int64_t out_w = 0, out_b = 0;
    std::vector<Entry> entries;  // parameter-vector order
    int64_t nparam = 0, naux = 0;
    // device memory
    Buf params, grads, mom1, mom2, pbf, aux;
    Buf xin, a, cat, eD, pool, c, d, y32, t32;       // forward activations
    Buf da, dcat, deD, dpool, dc, dd, dy32;         // gradients
    Buf wpart, bpart, lpart, loss_dev, hyper, scal, kpart;
    // the weight tensors whose data-gradient matrices Adam refreshes
    // (device AuxSeg table, sorted by parameter offset), and the host copy
    Buf segs;
    std::vector<AuxSeg> h_segs;
    int64_t aux_tiles = 0;   // transpose tiles over all weight tensors
    Buf amax;   // per-block maxima of absmax
    std::vector<int64_t> a_off, cat_off, pool_off, c_off, d_off;  // per level offsets (elements)
    int64_t wpart_max = 0, bpart_max = 0;
    // each weight gradient of a backward pass takes its own stretch of wpart
    // and bpart (cursors reset per pass), so that the second passes of all of
    // them run as one launch at the end of the pass: their arguments (fin),
    // the finish blocks before each (fin_begin), and the device copies
    int64_t wp_cursor = 0, bp_cursor = 0;
    std::vector<WgradArgs> fin, fin_dev_copy;
    std::vector<int64_t> fin_begin, fin_beg_copy;
    Buf fin_tab, fin_beg;
    int nblk0 = 0;
    // training run in progress (deblur_train_range): the next step of a
    // schedule of run_total steps at run_lr; run_next < 0 = none
    int32_t run_next = -1, run_total = 0;
    float run_lr = 0.f;
    // per-layer profiling
    bool prof = false;
    std::vector<ProfRec> prof_recs;
    std::vector<hipEvent_t> prof_events;
    size_t prof_used = 0;
};

namespace {

int set_err(deblur_net *n, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (n) n->err = buf;
    return code;
}

#define HCK(net, call)                                                                         \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return set_err(net, FWI_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));     \
    } while (0)

int alloc(deblur_net *n, Buf &b, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (b.bytes >= bytes) return FWI_OK;
    if (b.p) HCK(n, hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return set_err(n, FWI_ENOMEM, "device allocation of %zu bytes failed", bytes);
    }
    b.bytes = bytes;
    return FWI_OK;
}

void release(Buf &b)
{
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

template <class T>
T *P_(const Buf &b, int64_t off = 0)
{
    return static_cast<T *>(b.p) + off;
}

// ---- layout -----------------------------------------------------------------

ConvL add_conv(deblur_net *n, int cin, int cout, const char *name)
{
    ConvL L{cin, cout, n->nparam, 0, n->naux, {}};
    std::snprintf(L.name, sizeof L.name, "%s", name);
    n->entries.push_back({KW3, cin, cout, n->nparam, int64_t(cout) * cin * 9});
    n->nparam += int64_t(cout) * cin * 9;
    L.b = n->nparam;
    n->entries.push_back({KB, cin, cout, n->nparam, cout});
    n->nparam += cout;
    n->naux += int64_t(cout) * cin * 9;
    return L;
}

ConvL add_convt(deblur_net *n, int cin, int cout, const char *name)
{
    ConvL L{cin, cout, n->nparam, 0, n->naux, {}};
    std::snprintf(L.name, sizeof L.name, "%s", name);
    n->entries.push_back({KWT, cin, cout, n->nparam, int64_t(cin) * cout * 4});
    n->nparam += int64_t(cin) * cout * 4;
    L.b = n->nparam;
    n->entries.push_back({KB, cin, cout, n->nparam, cout});
    n->nparam += cout;
    n->naux += int64_t(cin) * cout * 4;
    return L;
}

void build_layout(deblur_net *n)
{
    const int D = n->D;
    n->C.resize(D + 1);
    n->H.resize(D + 1);
    n->W.resize(D + 1);
    n->P.resize(D + 1);
    for (int l = 0; l <= D; ++l) {
        n->C[l] = n->cfg.base_ch << l;
        n->H[l] = n->cfg.in_h >> l;
        n->W[l] = n->cfg.in_w >> l;
        n->P[l] = n->H[l] * n->W[l];
    }
    char nm[24];
    n->inc[0] = add_conv(n, 1, n->C[0], "inc.1");
    n->inc[1] = add_conv(n, n->C[0], n->C[0], "inc.2");
    n->down1.assign(D + 1, ConvL{});
    n->down2.assign(D + 1, ConvL{});
    n->upT.assign(D, ConvL{});
    n->up1.assign(D, ConvL{});
    n->up2.assign(D, ConvL{});
    for (int l = 1; l <= D; ++l) {
        std::snprintf(nm, sizeof nm, "down%d.1", l);
        n->down1[l] = add_conv(n, n->C[l - 1], n->C[l], nm);
        std::snprintf(nm, sizeof nm, "down%d.2", l);
        n->down2[l] = add_conv(n, n->C[l], n->C[l], nm);
    }
    for (int l = D - 1; l >= 0; --l) {
        std::snprintf(nm, sizeof nm, "up%d.T", l);
        n->upT[l] = add_convt(n, n->C[l + 1], n->C[l], nm);
        std::snprintf(nm, sizeof nm, "up%d.1", l);
        n->up1[l] = add_conv(n, 2 * n->C[l], n->C[l], nm);
        std::snprintf(nm, sizeof nm, "up%d.2", l);
        n->up2[l] = add_conv(n, n->C[l], n->C[l], nm);
    }
    n->out_w = n->nparam;
    n->entries.push_back({KW1, n->C[0], 1, n->nparam, n->C[0]});
    n->nparam += n->C[0];
    n->out_b = n->nparam;
    n->entries.push_back({KB, n->C[0], 1, n->nparam, 1});
    n->nparam += 1;
}

// output tile, pixels per split and split count of a weight-gradient
// reduction: the tile's height follows M (32, 64 or 128 rows), its width is
// 128 unless N is narrower; pixel splits (at least 256 pixels each) fill the
// GPU up to its resident workgroups
void wsplit(int M, int N, int P, int *nsplit, int *chunk, int *bm, int *bn)
{
    int tm = M <= 32 ? 32 : (M <= 64 ? 64 : 128);
    int tn = 128;
    if (N <= 64 || (tm == 64 && N < 128)) tm = 64, tn = 64;
    const int tiles = ((M + tm - 1) / tm) * ((N + tn - 1) / tn);
    // as many pixel splits as keep the grid within one round of resident
    // workgroups (two per CU for the 128-, 64- and 32-row tiles, four for 64 x
    // 64): a grid just past it leaves a second round of a few workgroups
    const int cap = tm == 64 && tn == 64 ? 1024 : 512;
    int ns = std::max(1, std::min(cap / tiles, std::max(1, P / 256)));
    int ch = (P + ns - 1) / ns;
    ch = ((ch + 63) / 64) * 64;
    ns = (P + ch - 1) / ch;
    *bm = tm;
    *bn = tn;
    *nsplit = ns;
    *chunk = ch;
}

int alloc_buffers(deblur_net *n)
{
    const int D = n->D;
    int rc;
    const size_t np = size_t(n->nparam);
    if ((rc = alloc(n, n->params, np * 4)) || (rc = alloc(n, n->grads, np * 4)) ||
        (rc = alloc(n, n->mom1, np * 4)) || (rc = alloc(n, n->mom2, np * 4)) ||
        (rc = alloc(n, n->pbf, np * 2)) || (rc = alloc(n, n->aux, size_t(n->naux) * 2)))
        return rc;
    int64_t sa = 0, sc = 0, sp = 0, scc = 0, sd = 0;
    n->a_off.assign(D + 1, 0);
    n->cat_off.assign(D + 1, 0);
    n->pool_off.assign(D + 1, 0);
    n->c_off.assign(D + 1, 0);
    n->d_off.assign(D + 1, 0);
    for (int l = 0; l <= D; ++l) {
        n->a_off[l] = sa;
        sa += int64_t(n->P[l]) * n->C[l];
        if (l < D) {
            n->cat_off[l] = sc;
            sc += int64_t(n->P[l]) * 2 * n->C[l];
            n->c_off[l] = scc;
            scc += int64_t(n->P[l]) * n->C[l];
            n->d_off[l] = sd;
            sd += int64_t(n->P[l]) * n->C[l];
        }
        if (l >= 1) {
            n->pool_off[l] = sp;
            sp += int64_t(n->P[l]) * n->C[l - 1];
        }
    }
    const int64_t eD = int64_t(n->P[D]) * n->C[D];
    const int64_t P0 = n->P[0];
    if ((rc = alloc(n, n->xin, size_t(P0) * 2)) || (rc = alloc(n, n->a, size_t(sa) * 2)) ||
        (rc = alloc(n, n->cat, size_t(sc) * 2)) || (rc = alloc(n, n->eD, size_t(eD) * 2)) ||
        (rc = alloc(n, n->pool, size_t(sp) * 2)) || (rc = alloc(n, n->c, size_t(scc) * 2)) ||
        (rc = alloc(n, n->d, size_t(sd) * 2)) || (rc = alloc(n, n->y32, size_t(P0) * 4)) ||
        (rc = alloc(n, n->t32, size_t(P0) * 4)) || (rc = alloc(n, n->da, size_t(sa) * 2)) ||
        (rc = alloc(n, n->dcat, size_t(sc) * 2)) || (rc = alloc(n, n->deD, size_t(eD) * 2)) ||
        (rc = alloc(n, n->dpool, size_t(sp) * 2)) || (rc = alloc(n, n->dc, size_t(scc) * 2)) ||
        (rc = alloc(n, n->dd, size_t(sd) * 2)) || (rc = alloc(n, n->dy32, size_t(P0) * 4)))
        return rc;
    // scratch of the weight- and bias-gradient reductions: one stretch per
    // layer of a backward pass (the sum over the layers)
    int64_t wmax = 0, bmax = 0;
    auto acc_w = [&](int M, int N, int P) {
        int ns, ch, bm, bn;
        wsplit(M, N, P, &ns, &ch, &bm, &bn);
        wmax += int64_t(ns) * M * N;
        bmax += int64_t(ns) * std::max(M, N);   // bias partials from A ([ns][M]) or B ([ns][N])
    };
    acc_w(n->inc[1].cout, 9 * n->inc[1].cin, n->P[0]);
    for (int l = 1; l <= D; ++l)
        for (const ConvL *L : {&n->down1[l], &n->down2[l]}) acc_w(L->cout, 9 * L->cin, n->P[l]);
    for (int l = 0; l < D; ++l) {
        for (const ConvL *L : {&n->up1[l], &n->up2[l]}) acc_w(L->cout, 9 * L->cin, n->P[l]);
        acc_w(n->upT[l].cin, 4 * n->upT[l].cout, n->P[l + 1]);
    }
    wmax += int64_t((P0 + 255) / 256) * (n->C[0] + 1);   // output-conv partials
    wmax += int64_t(512) * n->C[0] * 10;                  // input-layer partials
    n->wpart_max = wmax;
    if ((rc = alloc(n, n->kpart, size_t(kGemmSplitFloats) * 4))) return rc;
    n->bpart_max = bmax;
    n->nblk0 = int((P0 + 255) / 256);
    if ((rc = alloc(n, n->wpart, size_t(wmax) * 4)) || (rc = alloc(n, n->bpart, size_t(bmax) * 4)) ||
        (rc = alloc(n, n->lpart, size_t(std::max<int64_t>(n->nblk0 * int64_t(n->C[0] + 1), n->nblk0)) * 8)) ||
        (rc = alloc(n, n->scal, 64)) || (rc = alloc(n, n->amax, size_t(kAbsmaxBlocks) * 4)))
        return rc;
    return FWI_OK;
}

// ---- initialisation and parameter exchange -------------------------------------

uint64_t splitmix(uint64_t &s)
{
    uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

// default initialisation, in parameter-vector order and PyTorch layout:
// weights and biases uniform in +-1/sqrt(fan_in) (fan_in = Cin*9 for 3x3,
// Cout*4 for the transposed conv, C0 for the output conv)
std::vector<float> init_params(const deblur_net *n, uint64_t seed)
{
    std::vector<float> v(size_t(n->nparam));
    uint64_t s = seed;
    for (const Entry &e : n->entries) {
        double fan = 1;
        switch (e.kind) {
        case KW3: fan = e.cin * 9.0; break;
        case KWT: fan = e.cout * 4.0; break;
        case KW1: fan = e.cin; break;
        default: break;
        }
        if (e.kind == KB) {
            // fan of the weight just before it
            const Entry &w = *(&e - 1);
            fan = w.kind == KW3 ? w.cin * 9.0 : (w.kind == KWT ? w.cout * 4.0 : w.cin);
        }
        const double bound = 1.0 / std::sqrt(fan);
        for (int64_t i = 0; i < e.n; ++i) {
            const double u = double(splitmix(s) >> 11) * (1.0 / 9007199254740992.0);
            v[size_t(e.off + i)] = float((2.0 * u - 1.0) * bound);
        }
    }
    return v;
}

// PyTorch layout <-> internal layout (3x3: [co][tap][ci]; transposed conv:
// [ab][co][ci]); biases and the 1x1 conv are unchanged
void torch_to_internal(const deblur_net *n, const float *src, std::vector<float> &dst)
{
    dst.assign(size_t(n->nparam), 0.f);
    for (const Entry &e : n->entries) {
        const float *s = src + e.off;
        float *d = dst.data() + e.off;
        if (e.kind == KW3) {
            for (int co = 0; co < e.cout; ++co)
                for (int ci = 0; ci < e.cin; ++ci)
                    for (int t = 0; t < 9; ++t)
                        d[int64_t(co) * 9 * e.cin + int64_t(t) * e.cin + ci] = s[(int64_t(co) * e.cin + ci) * 9 + t];
        } else if (e.kind == KWT) {
            for (int ci = 0; ci < e.cin; ++ci)
                for (int co = 0; co < e.cout; ++co)
                    for (int ab = 0; ab < 4; ++ab)
                        d[(int64_t(ab) * e.cout + co) * e.cin + ci] = s[(int64_t(ci) * e.cout + co) * 4 + ab];
        } else {
            std::memcpy(d, s, size_t(e.n) * 4);
        }
    }
}

void internal_to_torch(const deblur_net *n, const float *src, float *dst)
{
    for (const Entry &e : n->entries) {
        const float *s = src + e.off;
        float *d = dst + e.off;
        if (e.kind == KW3) {
            for (int co = 0; co < e.cout; ++co)
                for (int ci = 0; ci < e.cin; ++ci)
                    for (int t = 0; t < 9; ++t)
                        d[(int64_t(co) * e.cin + ci) * 9 + t] = s[int64_t(co) * 9 * e.cin + int64_t(t) * e.cin + ci];
        } else if (e.kind == KWT) {
            for (int ci = 0; ci < e.cin; ++ci)
                for (int co = 0; co < e.cout; ++co)
                    for (int ab = 0; ab < 4; ++ab)
                        d[(int64_t(ci) * e.cout + co) * 4 + ab] = s[(int64_t(ab) * e.cout + co) * e.cin + ci];
        } else {
            std::memcpy(d, s, size_t(e.n) * 4);
        }
    }
}

// bf16 copies: the forward weight matrices and the data-gradient matrices
int refresh_weights(deblur_net *n, hipStream_t st)
{
    HCK(n, to_bf16(P_<float>(n->params), P_<bf16>(n->pbf), n->nparam, st));
    HCK(n, aux_from_pb(static_cast<const AuxSeg *>(n->segs.p), int32_t(n->h_segs.size()), n->aux_tiles,
                       P_<bf16>(n->pbf), P_<bf16>(n->aux), st));
    return FWI_OK;
}

int upload_params(deblur_net *n, hipStream_t st, const std::vector<float> &internal)
{
    HCK(n, hipMemcpyAsync(n->params.p, internal.data(), internal.size() * 4, hipMemcpyHostToDevice, st));
    HCK(n, hipStreamSynchronize(st));
    return refresh_weights(n, st);
}

// ---- layer launches ---------------------------------------------------------------

Gather conv_gather(const bf16 *src, int ld, int coff, int Cb, int H, int W)
{
    return Gather{src, ld, coff, Cb, H, W, H, W, 1, 3, -1, 9};
}

// per-layer profiling: events around one GEMM launch
int prof_begin(deblur_net *n, const char *name, int pass, int M, int N, int K, hipStream_t st)
{
    if (!n->prof) return FWI_OK;
    while (n->prof_used + 2 > n->prof_events.size()) {
        hipEvent_t e;
        HCK(n, hipEventCreate(&e));
        n->prof_events.push_back(e);
    }
    ProfRec r{name, pass, M, N, K, n->prof_events[n->prof_used], n->prof_events[n->prof_used + 1]};
    n->prof_used += 2;
    HCK(n, hipEventRecord(r.e0, st));
    n->prof_recs.push_back(r);
    return FWI_OK;
}

int prof_end(deblur_net *n, hipStream_t st)
{
    if (!n->prof) return FWI_OK;
    HCK(n, hipEventRecord(n->prof_recs.back().e1, st));
    return FWI_OK;
}

int conv_fwd(deblur_net *n, const ConvL &L, const bf16 *src, int ld, int coff, int lvl, bf16 *out, int out_ld,
             int out_coff, hipStream_t st)
{
    GemmArgs a{};
    a.kpart = P_<float>(n->kpart);
    a.kpart_cap = kGemmSplitFloats;
    a.M = L.cout;
    a.N = n->P[lvl];
    a.K = 9 * L.cin;
    a.A = P_<bf16>(n->pbf, L.w);
    a.lda = 9 * L.cin;
    a.g = conv_gather(src, ld, coff, L.cin, n->H[lvl], n->W[lvl]);
    a.out = out;
    a.out_ld = out_ld;
    a.out_coff = out_coff;
    a.Cout = L.cout;
    a.bias = P_<float>(n->params, L.b);
    a.act = 1;
    a.slope = n->cfg.leaky_slope;
    int rc = prof_begin(n, L.name, 0, a.M, a.N, a.K, st);
    if (rc) return rc;
    if (L.cin == 1 && ld == 1 && coff == 0 && L.cout % 8 == 0 && L.cout <= 1024 && out_ld % 8 == 0 &&
        out_coff % 8 == 0) {
        // the input layer: a direct convolution (K = 9 is too short for the matrix cores)
        HCK(n, conv1_fwd(src, n->H[lvl], n->W[lvl], a.A, a.bias, L.cout, 1, a.slope, out, out_ld, out_coff, st));
    } else {
        HCK(n, gemm(a, st));
    }
    return prof_end(n, st);
}

// dsrc = data gradient of a 3x3 conv given dz (the gradient at its
// pre-activation output)
int conv_dgrad(deblur_net *n, const ConvL &L, const bf16 *dz, int ldz, int zoff, int lvl, bf16 *dsrc, int ld,
               int coff, const bf16 *act_y, hipStream_t st)
{
    GemmArgs a{};
    a.kpart = P_<float>(n->kpart);
    a.kpart_cap = kGemmSplitFloats;
    a.M = L.cin;
    a.N = n->P[lvl];
    a.K = 9 * L.cout;
    a.A = P_<bf16>(n->aux, L.aux);
    a.lda = 9 * L.cout;
    a.g = conv_gather(dz, ldz, zoff, L.cout, n->H[lvl], n->W[lvl]);
    a.out = dsrc;
    a.out_ld = ld;
    a.out_coff = coff;
    a.Cout = L.cin;
    // act_y (the activated input of this layer, same layout as dsrc): the
    // result is the gradient at the pre-activation of the layer below
    a.act_y = act_y;
    a.act_ld = ld;
    a.act_coff = coff;
    a.slope = n->cfg.leaky_slope;
    int rc = prof_begin(n, L.name, 1, a.M, a.N, a.K, st);
    if (rc) return rc;
    HCK(n, gemm(a, st));
    return prof_end(n, st);
}

// the next stretch of the weight- / bias-gradient scratch (nullptr past the end)
float *take_w(deblur_net *n, int64_t floats)
{
    if (n->wp_cursor + floats > n->wpart_max) return nullptr;
    float *p = P_<float>(n->wpart, n->wp_cursor);
    n->wp_cursor += floats;
    return p;
}

float *take_b(deblur_net *n, int64_t floats)
{
    if (n->bp_cursor + floats > n->bpart_max) return nullptr;
    float *p = P_<float>(n->bpart, n->bp_cursor);
    n->bp_cursor += floats;
    return p;
}

void defer_finish(deblur_net *n, WgradArgs w)
{
    const int64_t cnt = wgrad_finish_count(w);
    if (cnt == 0) return;
    w.fin_groups = wgrad_finish_groups(w);
    const int64_t per = kFinishOutputs / w.fin_groups;
    if (n->fin_begin.empty()) n->fin_begin.push_back(0);
    n->fin.push_back(w);
    n->fin_begin.push_back(n->fin_begin.back() + (cnt + per - 1) / per);
}

// the deferred second passes of this backward pass, in one launch; the
// table is uploaded when it differs from the one on the device (the layer
// schedule is fixed, so in practice once)
int finish_weight_grads(deblur_net *n, hipStream_t st)
{
    if (n->fin.empty()) return FWI_OK;
    const size_t nf = n->fin.size();
    const bool same = n->fin_dev_copy.size() == nf &&
                      std::memcmp(n->fin_dev_copy.data(), n->fin.data(), nf * sizeof(WgradArgs)) == 0;
    if (!same) {
        int rc;
        if ((rc = alloc(n, n->fin_tab, nf * sizeof(WgradArgs))) ||
            (rc = alloc(n, n->fin_beg, (nf + 1) * sizeof(int64_t))))
            return rc;
        HCK(n, hipStreamSynchronize(st));   // the previous copies' host buffers are reused
        n->fin_dev_copy = n->fin;
        n->fin_beg_copy = n->fin_begin;
        HCK(n, hipMemcpyAsync(n->fin_tab.p, n->fin_dev_copy.data(), nf * sizeof(WgradArgs), hipMemcpyHostToDevice,
                              st));
        HCK(n, hipMemcpyAsync(n->fin_beg.p, n->fin_beg_copy.data(), (nf + 1) * sizeof(int64_t),
                              hipMemcpyHostToDevice, st));
    }
    HCK(n, wgrad_finish_all(static_cast<const WgradArgs *>(n->fin_tab.p), static_cast<const int64_t *>(n->fin_beg.p),
                            int32_t(nf), n->fin_begin.back(), st));
    return FWI_OK;
}

int conv_wgrad(deblur_net *n, const ConvL &L, const bf16 *dz, int ldz, int zoff, const bf16 *src, int ld, int coff,
               int lvl, hipStream_t st)
{
    WgradArgs w{};
    w.M = L.cout;
    w.N = 9 * L.cin;
    w.A = dz;
    w.lda = ldz;
    w.acoff = zoff;
    w.g = conv_gather(src, ld, coff, L.cin, n->H[lvl], n->W[lvl]);
    wsplit(w.M, w.N, n->P[lvl], &w.nsplit, &w.chunk, &w.bm, &w.bn);
    w.out = P_<float>(n->grads, L.w);
    w.ldm = 9 * L.cin;
    w.ldn = 1;
    w.bias_out = P_<float>(n->grads, L.b);
    int rc = prof_begin(n, L.name, 2, w.M, w.N, n->P[lvl], st);
    if (rc) return rc;
    if (L.cin == 1 && ld == 1 && coff == 0 && L.cout % 8 == 0 && L.cout <= 2048 && ldz % 8 == 0 && zoff % 8 == 0) {
        const int64_t cap = int64_t(512) * L.cout * 10;
        float *part = take_w(n, cap);
        if (!part) return set_err(n, FWI_EINVAL, "weight-gradient scratch exhausted");
        HCK(n, conv1_wgrad(dz, ldz, zoff, src, n->H[lvl], n->W[lvl], L.cout, part, cap, w.out, w.bias_out, st));
    } else {
        w.partial = take_w(n, int64_t(w.nsplit) * w.M * w.N);
        w.bias_partial = take_b(n, int64_t(w.nsplit) * std::max(w.M, w.N));
        if (!w.partial || !w.bias_partial) return set_err(n, FWI_EINVAL, "weight-gradient scratch exhausted");
        HCK(n, wgrad(w, st, true));
        defer_finish(n, w);
    }
    return prof_end(n, st);
}

// transposed conv of level l: src (level l+1, dense C_{l+1}) -> slice
// [C_l, 2C_l) of cat_l
int convt_fwd(deblur_net *n, int l, const bf16 *src, hipStream_t st)
{
    const ConvL &T = n->upT[l];
    GemmArgs a{};
    a.kpart = P_<float>(n->kpart);
    a.kpart_cap = kGemmSplitFloats;
    a.M = 4 * T.cout;
    a.N = n->P[l + 1];
    a.K = T.cin;
    a.A = P_<bf16>(n->pbf, T.w);
    a.lda = T.cin;
    a.g = Gather{src, T.cin, 0, T.cin, n->H[l + 1], n->W[l + 1], n->H[l + 1], n->W[l + 1], 1, 1, 0, 1};
    a.out = P_<bf16>(n->cat, n->cat_off[l]);
    a.out_ld = 2 * n->C[l];
    a.out_coff = n->C[l];
    a.Cout = T.cout;
    a.scatter = 1;
    a.Ho = n->H[l];
    a.Wo = n->W[l];
    a.bias = P_<float>(n->params, T.b);
    int rc = prof_begin(n, T.name, 0, a.M, a.N, a.K, st);
    if (rc) return rc;
    HCK(n, gemm(a, st));
    return prof_end(n, st);
}

int convt_bwd(deblur_net *n, int l, const bf16 *src, bf16 *dsrc, hipStream_t st)
{
    const ConvL &T = n->upT[l];
    const bf16 *du = P_<bf16>(n->dcat, n->cat_off[l]);
    const Gather gu{du, 2 * n->C[l], n->C[l], T.cout, n->H[l], n->W[l], n->H[l + 1], n->W[l + 1], 2, 2, 0, 4};
    WgradArgs w{};
    w.M = T.cin;
    w.N = 4 * T.cout;
    w.A = src;
    w.lda = T.cin;
    w.acoff = 0;
    w.g = gu;
    wsplit(w.M, w.N, n->P[l + 1], &w.nsplit, &w.chunk, &w.bm, &w.bn);
    w.partial = take_w(n, int64_t(w.nsplit) * w.M * w.N);
    w.out = P_<float>(n->grads, T.w);
    w.ldm = 1;
    w.ldn = T.cin;
    // the bias gradient is the sum of the gathered output gradient
    w.bias_partial = take_b(n, int64_t(w.nsplit) * std::max(w.M, w.N));
    w.bias_out = P_<float>(n->grads, T.b);
    w.bias_from_b = 1;
    if (!w.partial || !w.bias_partial) return set_err(n, FWI_EINVAL, "weight-gradient scratch exhausted");
    int rc = prof_begin(n, T.name, 2, w.M, w.N, n->P[l + 1], st);
    if (rc) return rc;
    HCK(n, wgrad(w, st, true));
    defer_finish(n, w);
    if ((rc = prof_end(n, st))) return rc;
    GemmArgs a{};
    a.kpart = P_<float>(n->kpart);
    a.kpart_cap = kGemmSplitFloats;
    a.M = T.cin;
    a.N = n->P[l + 1];
    a.K = 4 * T.cout;
    a.A = P_<bf16>(n->aux, T.aux);
    a.lda = 4 * T.cout;
    a.g = gu;
    a.out = dsrc;
    a.out_ld = T.cin;
    a.Cout = T.cin;
    // src is the activated output of the layer below (dense, T.cin channels)
    a.act_y = src;
    a.act_ld = T.cin;
    a.act_coff = 0;
    a.slope = n->cfg.leaky_slope;
    if ((rc = prof_begin(n, T.name, 1, a.M, a.N, a.K, st))) return rc;
    HCK(n, gemm(a, st));
    return prof_end(n, st);
}

// forward of the padded, normalised input in xin (bf16) to y32 (FP32)
int forward(deblur_net *n, hipStream_t st)
{
    const int D = n->D;
    int rc;
    bf16 *cat = P_<bf16>(n->cat), *a = P_<bf16>(n->a), *pl = P_<bf16>(n->pool);
    bf16 *c = P_<bf16>(n->c), *d = P_<bf16>(n->d), *eD = P_<bf16>(n->eD);
    // input block
    if ((rc = conv_fwd(n, n->inc[0], P_<bf16>(n->xin), 1, 0, 0, a + n->a_off[0], n->C[0], 0, st))) return rc;
    if ((rc = conv_fwd(n, n->inc[1], a + n->a_off[0], n->C[0], 0, 0, cat + n->cat_off[0], 2 * n->C[0], 0, st)))
        return rc;
    // encoder
    for (int l = 1; l <= D; ++l) {
        HCK(n, pool_fwd(cat + n->cat_off[l - 1], 2 * n->C[l - 1], 0, n->C[l - 1], n->H[l - 1], n->W[l - 1],
                        pl + n->pool_off[l], st));
        if ((rc = conv_fwd(n, n->down1[l], pl + n->pool_off[l], n->C[l - 1], 0, l, a + n->a_off[l], n->C[l], 0, st)))
            return rc;
        bf16 *eo = l < D ? cat + n->cat_off[l] : eD;
        const int eld = l < D ? 2 * n->C[l] : n->C[l];
        if ((rc = conv_fwd(n, n->down2[l], a + n->a_off[l], n->C[l], 0, l, eo, eld, 0, st))) return rc;
    }
    // decoder
    for (int l = D - 1; l >= 0; --l) {
        const bf16 *src = l == D - 1 ? eD : d + n->d_off[l + 1];
        if ((rc = convt_fwd(n, l, src, st))) return rc;
        if ((rc = conv_fwd(n, n->up1[l], cat + n->cat_off[l], 2 * n->C[l], 0, l, c + n->c_off[l], n->C[l], 0, st)))
            return rc;
        if ((rc = conv_fwd(n, n->up2[l], c + n->c_off[l], n->C[l], 0, l, d + n->d_off[l], n->C[l], 0, st))) return rc;
    }
    HCK(n, outc_fwd(d + n->d_off[0], n->C[0], n->P[0], P_<float>(n->params, n->out_w),
                    P_<float>(n->params, n->out_b), P_<float>(n->y32), st));
    return FWI_OK;
}

// loss (into loss_slot, FP64 device, and its FP32 copy) and all parameter
// gradients for target t32
int backward(deblur_net *n, hipStream_t st, double *loss_slot)
{
    const int D = n->D;
    const float slope = n->cfg.leaky_slope;
    int rc;
    bf16 *cat = P_<bf16>(n->cat), *a = P_<bf16>(n->a), *pl = P_<bf16>(n->pool);
    bf16 *c = P_<bf16>(n->c), *d = P_<bf16>(n->d), *eD = P_<bf16>(n->eD);
    bf16 *dcat = P_<bf16>(n->dcat), *da = P_<bf16>(n->da), *dpl = P_<bf16>(n->dpool);
    bf16 *dc = P_<bf16>(n->dc), *dd = P_<bf16>(n->dd), *deD = P_<bf16>(n->deD);
    const int P0 = n->P[0], C0 = n->C[0];
    double *lpart = P_<double>(n->lpart);
    HCK(n, mse(P_<float>(n->y32), P_<float>(n->t32), P0, lpart, n->nblk0, P_<float>(n->dy32), st));
    HCK(n, sum_partials_d(lpart, n->nblk0, loss_slot, 1.0f / float(P0), nullptr, st));
    n->wp_cursor = n->bp_cursor = 0;
    n->fin.clear();
    n->fin_begin.clear();
    float *wp = take_w(n, int64_t(n->nblk0) * (C0 + 1));
    if (!wp) return set_err(n, FWI_EINVAL, "weight-gradient scratch exhausted");
    // Every activation derivative is folded into the kernel that produces the
    // gradient it scales: the output convolution's backward (dd_0), the data
    // gradients whose input was activated (act_y), and the pooling adjoint
    // that completes a skip connection's gradient (after its accumulation).
    HCK(n, outc_bwd(d + n->d_off[0], C0, P0, P_<float>(n->params, n->out_w), P_<float>(n->dy32), dd + n->d_off[0], wp,
                    n->nblk0, slope, st));
    HCK(n, outc_wgrad_reduce(wp, C0, n->nblk0, P_<float>(n->grads, n->out_w), P_<float>(n->grads, n->out_b), st));
    // decoder, level 0 up to D-1
    for (int l = 0; l < D; ++l) {
        const int Cl = n->C[l];
        bf16 *ddl = dd + n->d_off[l], *dcl = dc + n->c_off[l];
        if ((rc = conv_wgrad(n, n->up2[l], ddl, Cl, 0, c + n->c_off[l], Cl, 0, l, st))) return rc;
        if ((rc = conv_dgrad(n, n->up2[l], ddl, Cl, 0, l, dcl, Cl, 0, c + n->c_off[l], st))) return rc;
        if ((rc = conv_wgrad(n, n->up1[l], dcl, Cl, 0, cat + n->cat_off[l], 2 * Cl, 0, l, st))) return rc;
        if ((rc = conv_dgrad(n, n->up1[l], dcl, Cl, 0, l, dcat + n->cat_off[l], 2 * Cl, 0, nullptr, st))) return rc;
        const bf16 *src = l == D - 1 ? eD : d + n->d_off[l + 1];
        bf16 *dsrc = l == D - 1 ? deD : dd + n->d_off[l + 1];
        if ((rc = convt_bwd(n, l, src, dsrc, st))) return rc;
    }
    // encoder, level D down to 1
    for (int l = D; l >= 1; --l) {
        const int Cl = n->C[l];
        bf16 *de = l < D ? dcat + n->cat_off[l] : deD;
        const int eld = l < D ? 2 * Cl : Cl;
        bf16 *dal = da + n->a_off[l];
        if ((rc = conv_wgrad(n, n->down2[l], de, eld, 0, a + n->a_off[l], Cl, 0, l, st))) return rc;
        if ((rc = conv_dgrad(n, n->down2[l], de, eld, 0, l, dal, Cl, 0, a + n->a_off[l], st))) return rc;
        const int Cp = n->C[l - 1];
        if ((rc = conv_wgrad(n, n->down1[l], dal, Cl, 0, pl + n->pool_off[l], Cp, 0, l, st))) return rc;
        if ((rc = conv_dgrad(n, n->down1[l], dal, Cl, 0, l, dpl + n->pool_off[l], Cp, 0, nullptr, st))) return rc;
        HCK(n, pool_bwd(dpl + n->pool_off[l], Cp, n->H[l - 1], n->W[l - 1], dcat + n->cat_off[l - 1], 2 * Cp, 0, 1,
                        cat + n->cat_off[l - 1], slope, st));
    }
    // input block
    bf16 *de0 = dcat + n->cat_off[0];
    if ((rc = conv_wgrad(n, n->inc[1], de0, 2 * C0, 0, a + n->a_off[0], C0, 0, 0, st))) return rc;
    bf16 *da0 = da + n->a_off[0];
    if ((rc = conv_dgrad(n, n->inc[1], de0, 2 * C0, 0, 0, da0, C0, 0, a + n->a_off[0], st))) return rc;
    if ((rc = conv_wgrad(n, n->inc[0], da0, C0, 0, P_<bf16>(n->xin), 1, 0, 0, st))) return rc;
    return finish_weight_grads(n, st);
}

int check_ctx(deblur_net *n, fwi_ctx *ctx, hipStream_t *st)
{
    if (!n || !ctx) return FWI_EINVAL;
    n->err.clear();
    if (fwi::ctx_device(ctx) != n->device)
        return set_err(n, FWI_EINVAL, "context device %d differs from the network's %d", fwi::ctx_device(ctx),
                       n->device);
    HCK(n, hipSetDevice(n->device));
    *st = fwi::ctx_stream(ctx);
    return FWI_OK;
}

int check_image(deblur_net *n, int nz, int nx, int *py, int *px)
{
    if (nz < 1 || nx < 1 || nz > n->cfg.in_h || nx > n->cfg.in_w)
        return set_err(n, FWI_EINVAL, "image %dx%d does not fit the %dx%d network grid", nz, nx, n->cfg.in_h,
                       n->cfg.in_w);
    // padding above / left rounded down; an odd remainder goes below / right
    *py = (n->cfg.in_h - nz) / 2;
    *px = (n->cfg.in_w - nx) / 2;
    const int pb = n->cfg.in_h - nz - *py, pr = n->cfg.in_w - nx - *px;
    if ((pb > 0 && pb >= nz) || (pr > 0 && pr >= nx))
        return set_err(n, FWI_EINVAL, "reflect padding wider than the image");
    return FWI_OK;
}

}  // namespace

extern "C" {

int deblur_create(fwi_ctx *ctx, const deblur_cfg *cfg, uint64_t seed, deblur_net **out)
{
    if (!ctx || !cfg || !out) return FWI_EINVAL;
    *out = nullptr;
    if (cfg->depth < 1 || cfg->depth > 6 || cfg->base_ch < 8 || cfg->base_ch % 8 || cfg->base_ch > 1024 ||
        cfg->in_h < 1 || cfg->in_w < 1 || cfg->in_h % (1 << cfg->depth) || cfg->in_w % (1 << cfg->depth) ||
        !(cfg->leaky_slope >= 0.f && cfg->leaky_slope < 1.f))
        return FWI_EINVAL;
    deblur_net *n = new deblur_net();
    n->cfg = *cfg;
    n->D = cfg->depth;
    n->device = fwi::ctx_device(ctx);
    if (hipSetDevice(n->device) != hipSuccess) {
        delete n;
        return FWI_EHIP;
    }
    build_layout(n);
    int rc = alloc_buffers(n);
    if (rc == FWI_OK) {
        // weight tensors in parameter order with their data-gradient matrices
        // (laid out in the same order)
        int64_t aux = 0;
        for (const Entry &e : n->entries) {
            if (e.kind != KW3 && e.kind != KWT) continue;
            if (e.kind == KW3 && e.cin == 1) {   // the input layer: no data gradient is formed
                aux += e.n;
                continue;
            }
            const int R = e.kind == KW3 ? e.cout : 4 * e.cout, C = e.kind == KW3 ? 9 * e.cin : e.cin;
            n->h_segs.push_back(AuxSeg{e.off, e.n, aux, n->aux_tiles, e.kind == KW3 ? 0 : 1, e.cin, e.cout, 0});
            aux += e.n;
            n->aux_tiles += int64_t((R + 63) / 64) * ((C + 63) / 64);
        }
        rc = alloc(n, n->segs, n->h_segs.size() * sizeof(AuxSeg));
        if (rc == FWI_OK && hipMemcpyAsync(n->segs.p, n->h_segs.data(), n->h_segs.size() * sizeof(AuxSeg),
                                           hipMemcpyHostToDevice, fwi::ctx_stream(ctx)) != hipSuccess)
            rc = set_err(n, FWI_EHIP, "upload of the weight table failed");
    }
    if (rc == FWI_OK) {
        std::vector<float> v = init_params(n, seed), internal;
        torch_to_internal(n, v.data(), internal);
        rc = upload_params(n, fwi::ctx_stream(ctx), internal);
    }
    if (rc != FWI_OK) {
        deblur_destroy(n);
        return rc;
    }
    *out = n;
    return FWI_OK;
}

void deblur_destroy(deblur_net *n)
{
    if (!n) return;
    (void)hipSetDevice(n->device);
    (void)hipDeviceSynchronize();
    for (Buf *b : {&n->params, &n->grads, &n->mom1, &n->mom2, &n->pbf, &n->aux, &n->xin, &n->a, &n->cat, &n->eD,
                   &n->pool, &n->c, &n->d, &n->y32, &n->t32, &n->da, &n->dcat, &n->deD, &n->dpool, &n->dc, &n->dd,
                   &n->dy32, &n->wpart, &n->bpart, &n->lpart, &n->loss_dev, &n->hyper, &n->scal, &n->kpart,
                   &n->segs, &n->fin_tab, &n->fin_beg, &n->amax})
        release(*b);
    for (hipEvent_t e : n->prof_events) (void)hipEventDestroy(e);
    delete n;
}

const char *deblur_last_error(const deblur_net *n)
{
    return n ? n->err.c_str() : "NULL network";
}

int deblur_num_params(const deblur_net *n, int64_t *np)
{
    if (!n || !np) return FWI_EINVAL;
    *np = n->nparam;
    return FWI_OK;
}

int deblur_set_params(fwi_ctx *ctx, deblur_net *n, const float *params)
{
    if (n) n->run_next = -1;   // new weights end a training run
    hipStream_t st;
    int rc = check_ctx(n, ctx, &st);
    if (rc) return rc;
    if (!params) return set_err(n, FWI_EINVAL, "params is NULL");
    std::vector<float> internal;
    torch_to_internal(n, params, internal);
    return upload_params(n, st, internal);
}

int deblur_get_params(fwi_ctx *ctx, const deblur_net *cn, float *params)
{
    deblur_net *n = const_cast<deblur_net *>(cn);
    hipStream_t st;
    int rc = check_ctx(n, ctx, &st);
    if (rc) return rc;
    if (!params) return set_err(n, FWI_EINVAL, "params is NULL");
    std::vector<float> internal(size_t(n->nparam));
    HCK(n, hipMemcpyAsync(internal.data(), n->params.p, internal.size() * 4, hipMemcpyDeviceToHost, st));
    HCK(n, hipStreamSynchronize(st));
    internal_to_torch(n, internal.data(), params);
    return FWI_OK;
}

int deblur_reset(fwi_ctx *ctx, deblur_net *n, uint64_t seed)
{
    if (n) n->run_next = -1;   // new weights end a training run
    hipStream_t st;
    int rc = check_ctx(n, ctx, &st);
    if (rc) return rc;
    std::vector<float> v = init_params(n, seed), internal;
    torch_to_internal(n, v.data(), internal);
    return upload_params(n, st, internal);
}

int deblur_forward_raw(fwi_ctx *ctx, deblur_net *n, const float *x, float *y)
{
    hipStream_t st;
    int rc = check_ctx(n, ctx, &st);
    if (rc) return rc;
    if (!x || !y) return set_err(n, FWI_EINVAL, "NULL image");
    const int64_t P0 = n->P[0];
    HCK(n, to_bf16(x, P_<bf16>(n->xin), P0, st));
    if ((rc = forward(n, st))) return rc;
    HCK(n, hipMemcpyAsync(y, n->y32.p, size_t(P0) * 4, hipMemcpyDeviceToDevice, st));
    return FWI_OK;
}

int deblur_grad_raw(fwi_ctx *ctx, deblur_net *n, const float *x, const float *t, double *loss, float *grads)
{
    hipStream_t st;
    int rc = check_ctx(n, ctx, &st);
    if (rc) return rc;
    if (!x || !t) return set_err(n, FWI_EINVAL, "NULL image");
    const int64_t P0 = n->P[0];
    if ((rc = alloc(n, n->loss_dev, 8))) return rc;
    HCK(n, to_bf16(x, P_<bf16>(n->xin), P0, st));
    HCK(n, hipMemcpyAsync(n->t32.p, t, size_t(P0) * 4, hipMemcpyDeviceToDevice, st));
    if ((rc = forward(n, st)) || (rc = backward(n, st, P_<double>(n->loss_dev)))) return rc;
    double l = 0;
    HCK(n, hipMemcpyAsync(&l, n->loss_dev.p, 8, hipMemcpyDeviceToHost, st));
    std::vector<float> internal(size_t(n->nparam));
    HCK(n, hipMemcpyAsync(internal.data(), n->grads.p, internal.size() * 4, hipMemcpyDeviceToHost, st));
    HCK(n, hipStreamSynchronize(st));
    if (loss) *loss = l;
    if (grads) internal_to_torch(n, internal.data(), grads);
    return FWI_OK;
}

int deblur_train_range(fwi_ctx *ctx, deblur_net *n, const float *x, const float *y, int32_t nz, int32_t nx,
                       int32_t first, int32_t count, int32_t total, float lr_max, float *loss_hist)
{
    hipStream_t st;
    int rc = check_ctx(n, ctx, &st);
    if (rc) return rc;
    if (!x || !y) return set_err(n, FWI_EINVAL, "NULL image");
    if (first < 0 || count < 0 || total < 0 || int64_t(first) + count > total || !(lr_max >= 0.f))
        return set_err(n, FWI_EINVAL, "bad step range %d + %d of %d or learning rate", first, count, total);
    if (first > 0 && (n->run_next != first || n->run_total != total || n->run_lr != lr_max))
        return set_err(n, FWI_ESTATE, "step %d does not continue the network's training run", first);
    int py, px;
    if ((rc = check_image(n, nz, nx, &py, &px))) return rc;
    if (count == 0) return FWI_OK;
    n->run_next = -1;   // until this call has completed
    const int H = n->cfg.in_h, W = n->cfg.in_w;
    float *scal = P_<float>(n->scal);  // [0] max|x|, [1] max|y|
    if ((rc = alloc(n, n->loss_dev, size_t(count) * 8)) || (rc = alloc(n, n->hyper, size_t(count) * 3 * 4)))
        return rc;
    HCK(n, absmax(x, int64_t(nz) * nx, scal, P_<float>(n->amax), st));
    HCK(n, absmax(y, int64_t(nz) * nx, scal + 1, P_<float>(n->amax), st));
    HCK(n, pad_norm(x, nz, nx, H, W, py, px, scal, P_<bf16>(n->xin), nullptr, st));
    HCK(n, pad_norm(y, nz, nx, H, W, py, px, scal + 1, nullptr, P_<float>(n->t32), st));
    // cosine-annealed learning rate (over the run's total steps) and the Adam
    // bias corrections of each step
    std::vector<float> hyper(size_t(count) * 3);
    for (int i = 0; i < count; ++i) {
        const int t = first + i;
        hyper[3 * i] = float(lr_max * 0.5 * (1.0 + std::cos(M_PI * double(t) / double(total))));
        hyper[3 * i + 1] = float(1.0 - std::pow(double(kBeta1), t + 1));
        hyper[3 * i + 2] = float(1.0 - std::pow(double(kBeta2), t + 1));
    }
    HCK(n, hipMemcpyAsync(n->hyper.p, hyper.data(), hyper.size() * 4, hipMemcpyHostToDevice, st));
    if (first == 0) {
        HCK(n, fill_f(P_<float>(n->mom1), n->nparam, 0.f, st));
        HCK(n, fill_f(P_<float>(n->mom2), n->nparam, 0.f, st));
    }
    for (int i = 0; i < count; ++i) {
        if ((rc = forward(n, st)) || (rc = backward(n, st, P_<double>(n->loss_dev, i)))) return rc;
        // the update writes the bf16 weights; the data-gradient matrices follow
        HCK(n, adam(P_<float>(n->params), P_<float>(n->grads), P_<float>(n->mom1), P_<float>(n->mom2),
                    P_<bf16>(n->pbf), n->nparam, P_<float>(n->hyper, 3 * i), kBeta1, kBeta2, kEps, st));
        HCK(n, aux_from_pb(static_cast<const AuxSeg *>(n->segs.p), int32_t(n->h_segs.size()), n->aux_tiles,
                           P_<bf16>(n->pbf), P_<bf16>(n->aux), st));
    }
    std::vector<double> lh(static_cast<size_t>(count));
    HCK(n, hipMemcpyAsync(lh.data(), n->loss_dev.p, lh.size() * 8, hipMemcpyDeviceToHost, st));
    HCK(n, hipStreamSynchronize(st));
    if (loss_hist)
        for (int i = 0; i < count; ++i) loss_hist[i] = float(lh[size_t(i)]);
    if (first + count < total) {
        n->run_next = first + count;
        n->run_total = total;
        n->run_lr = lr_max;
    }
    return FWI_OK;
}

int deblur_train(fwi_ctx *ctx, deblur_net *n, const float *x, const float *y, int32_t nz, int32_t nx, int32_t steps,
                 float lr_max, float *loss_hist)
{
    if (steps < 0) return n ? set_err(n, FWI_EINVAL, "bad steps or learning rate") : FWI_EINVAL;
    return deblur_train_range(ctx, n, x, y, nz, nx, 0, steps, steps, lr_max, loss_hist);
}

int deblur_apply(fwi_ctx *ctx, deblur_net *n, const float *x, int32_t nz, int32_t nx, float *y)
{
    hipStream_t st;
    int rc = check_ctx(n, ctx, &st);
    if (rc) return rc;
    if (!x || !y) return set_err(n, FWI_EINVAL, "NULL image");
    int py, px;
    if ((rc = check_image(n, nz, nx, &py, &px))) return rc;
    const int H = n->cfg.in_h, W = n->cfg.in_w;
    float *scal = P_<float>(n->scal);
    HCK(n, absmax(x, int64_t(nz) * nx, scal, P_<float>(n->amax), st));
    HCK(n, pad_norm(x, nz, nx, H, W, py, px, scal, P_<bf16>(n->xin), nullptr, st));
    if ((rc = forward(n, st))) return rc;
    HCK(n, crop_scale(P_<float>(n->y32), H, W, py, px, nz, nx, scal, y, st));
    return FWI_OK;
}

int deblur_set_profiling(deblur_net *n, int enable)
{
    if (!n) return FWI_EINVAL;
    n->prof = enable != 0;
    if (n->prof) {
        n->prof_recs.clear();
        n->prof_used = 0;
    }
    return FWI_OK;
}

int deblur_layer_stats(fwi_ctx *ctx, deblur_net *n, deblur_layer_stat *out, int32_t max, int32_t *count)
{
    if (!n || !count || (max > 0 && !out)) return FWI_EINVAL;
    hipStream_t st;
    int rc = check_ctx(n, ctx, &st);
    if (rc) return rc;
    HCK(n, hipStreamSynchronize(st));
    std::vector<deblur_layer_stat> agg;
    for (const ProfRec &r : n->prof_recs) {
        float ms = 0.f;
        HCK(n, hipEventElapsedTime(&ms, r.e0, r.e1));
        deblur_layer_stat *s = nullptr;
        for (auto &a : agg)
            if (a.pass == r.pass && std::strncmp(a.name, r.name, sizeof a.name) == 0) s = &a;
        if (!s) {
            agg.push_back(deblur_layer_stat{});
            s = &agg.back();
            std::snprintf(s->name, sizeof s->name, "%s", r.name);
            s->pass = r.pass;
            s->M = r.M;
            s->N = r.N;
            s->K = r.K;
        }
        s->calls += 1;
        s->flops += 2.0 * double(r.M) * r.N * r.K;
        s->ms += ms;
    }
    const int32_t k = int32_t(std::min<size_t>(agg.size(), size_t(std::max(max, 0))));
    for (int32_t i = 0; i < k; ++i) out[i] = agg[i];
    *count = int32_t(agg.size());
    return FWI_OK;
}

int deblur_save(fwi_ctx *ctx, const deblur_net *cn, const char *path)
{
    deblur_net *n = const_cast<deblur_net *>(cn);
    if (!path) return set_err(n, FWI_EINVAL, "NULL path");
    std::vector<float> v(size_t(n ? n->nparam : 0));
    int rc = deblur_get_params(ctx, n, v.data());
    if (rc) return rc;
    FILE *f = std::fopen(path, "wb");
    if (!f) return set_err(n, FWI_EINVAL, "cannot open %s", path);
    const uint32_t magic = kMagic;
    const int64_t np = n->nparam;
    bool ok = std::fwrite(&magic, 4, 1, f) == 1 && std::fwrite(&n->cfg, sizeof(deblur_cfg), 1, f) == 1 &&
              std::fwrite(&np, 8, 1, f) == 1 && std::fwrite(v.data(), 4, v.size(), f) == v.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? FWI_OK : set_err(n, FWI_EINVAL, "write to %s failed", path);
}

int deblur_load(fwi_ctx *ctx, deblur_net *n, const char *path)
{
    if (!n || !path) return FWI_EINVAL;
    FILE *f = std::fopen(path, "rb");
    if (!f) return set_err(n, FWI_EINVAL, "cannot open %s", path);
    uint32_t magic = 0;
    deblur_cfg cfg{};
    int64_t np = 0;
    bool ok = std::fread(&magic, 4, 1, f) == 1 && std::fread(&cfg, sizeof cfg, 1, f) == 1 &&
              std::fread(&np, 8, 1, f) == 1;
    ok = ok && magic == kMagic && np == n->nparam && std::memcmp(&cfg, &n->cfg, sizeof cfg) == 0;
    std::vector<float> v(size_t(n->nparam));
    ok = ok && std::fread(v.data(), 4, v.size(), f) == v.size();
    std::fclose(f);
    if (!ok) return set_err(n, FWI_EINVAL, "%s is not a checkpoint of this network", path);
    return deblur_set_params(ctx, n, v.data());
}

}  // extern "C"
