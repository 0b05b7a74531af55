// C ABI of libfwi.so (declared in include/fwi.h): argument checks, the
// per-call plan (shot layout, wave table, receiver tables), the scratch
// pool, the checkpointed adjoint sweeps, and kernel timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/fwi.h"
#include "internal.h"

using namespace fwi;

namespace {

constexpr double kCflLimit = 0.55;     // 2D 8th-order leapfrog limit is 0.5546
constexpr double kDefaultBudgetFrac = 0.7;  // of device memory, for D^n history + checkpoints
constexpr int64_t kFreeMargin = int64_t(4) << 30;  // left free when sizing the history
// Static device scratch of the allocation-free entry points (per device, held
// until the process ends).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kDefaultCw = 2;          // tiling used when autotuning is off
constexpr int kDefaultRows = 32;
constexpr int kDefaultTb = 1;
constexpr int kDefaultPd = 2;

// 8th-order central second-derivative weights (Fornberg 1988).
constexpr double kC8[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct Plan {
    // grid
    int nz = 0, nx = 0, nb = 0, NZ = 0, nt_max = 0, S = 0;
    int top = 0;                  // padded rows above physical row 0
    bool free_surface = false;    // pressure-free top surface (no top sponge)
    bool pml = false;             // perfectly matched layer in the padding (nb > 0)
    bool relative = false;        // Born perturbations and images per dV / V
    float h = 0, dt = 0, v_ref = 0, R = 0;
    int ckpt_every = 0;
    // shots in slot order (record length decreasing)
    std::vector<int> order;              // slot -> caller's shot index
    std::vector<ShotDesc> shots;
    std::vector<int> slot_nt;
    // receiver cells of every slot: ((row, col), q), sorted by row then col
    std::vector<std::vector<std::pair<std::pair<int, int>, int>>> slot_cells;
    // unique receiver cells
    int Q = 0;
    std::vector<int32_t> q_nt, q_rptr;
    std::vector<int64_t> q_roff;
    std::vector<float> q_rw;             // weight of each q_roff entry (1 on the grid)
    // receivers off the grid: each combines up to four cells (CSR per receiver)
    bool offgrid = false;
    int nrec = 0;
    std::vector<int32_t> r_cptr, r_cq, r_nt;
    std::vector<float> r_cw;
    std::vector<int64_t> r_off;
    std::vector<float> wav;
    int64_t field_floats = 0;  // one wavefield buffer, all shots
    int64_t img_floats = 0;    // one image / D slot, all shots
    int64_t data_size = 0;     // packed data samples
    double updates_per_field_pass = 0;
    std::vector<char> key;     // serialized inputs (plan cache)

    int active_slots(int n) const
    {
        // slots are sorted by decreasing nt: those with nt > n form a prefix
        int lo = 0, hi = S;
        while (lo < hi) {
            const int mid = (lo + hi) / 2;
            if (slot_nt[mid] > n) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    }
};

// Wave table of one tiling: strips of 64*cw columns, runs of `rows` rows.
struct Tiling {
    int cw = 0, rows = 0, tb = 0;  // columns per lane, rows per wave, time levels per launch
    int pd = 1;                    // one level per launch: rows prefetched ahead
    std::vector<WaveDesc> waves;
    std::vector<RecRow> rrows;
    std::vector<int32_t> rmap;
    std::vector<int> prefix;  // waves of slots [0, k)
    DevBuf d_waves, d_rrows, d_rmap;
    // two levels per launch: the one-level table over the same strip width,
    // for the single step a range of odd length ends with (the two-level
    // table's strips overlap by the 4-column halos and its receiver maps
    // start 4 columns left of a strip, which the one-level kernel does not)
    std::vector<WaveDesc> waves1;
    std::vector<RecRow> rrows1;
    std::vector<int32_t> rmap1;
    std::vector<int> prefix1;
    DevBuf d_waves1, d_rrows1, d_rmap1;
    void release_all();
};

// tiling classes: forward, adjoint, joint Born (one level per launch),
// scattered field from a stored history
enum KClass { K_FWD = 0, K_ADJ = 1, K_BORN = 2, K_SCAT = 3, K_OTHER = 4 };
constexpr int kClasses = 4;
// classes whose kernels advance one time level per launch
constexpr bool one_level(int k) { return k == K_BORN; }

// The two newest time levels of a sweep and two spare buffers. A one-level
// launch overwrites `prev` in place; a two-level launch writes the spares.
struct Fields {
    float *prev, *cur, *s0, *s1;
    // perfectly matched layer: the field's edge fields (x, z) at the previous
    // level and the buffers their next level goes to
    float *px = nullptr, *pz = nullptr, *qx = nullptr, *qz = nullptr;
};

// A time loop captured into a HIP graph: the key serializes every input the
// loop's launches depend on; `delta` holds the statistics one run adds and
// `after` the field rotation it leaves.
struct GraphEntry {
    std::vector<char> key;
    hipGraphExec_t exec = nullptr;
    fwi_stats delta{};
    Fields after{};
    uint64_t used = 0;
    size_t nodes = 0;
};
// captured loops kept per context: bounded by their total kernel nodes (a
// few hundred bytes of host memory each)
constexpr size_t kGraphNodeBudget = 400000;

}  // namespace

// The scratch of the allocation-free entry points. In host code this name is
// a stand-in, not a device address: the address of each device's copy is
// looked up once per device (scratch_address) and only that is used.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

struct fwi_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int64_t budget = 0;
    int ckpt_slots = -1;          // forced snapshot slots of the adjoint sweeps (-1: from the budget)
    bool profiling = false;
    fwi_stats stats{};
    Plan plan;
    bool plan_valid = false;
    // device copies of the plan tables
    DevBuf d_shots, d_qnt, d_qrptr, d_qroff, d_wav;
    DevBuf d_qrw, d_rcptr, d_rcq, d_rnt, d_rcw, d_roff;   // off-grid receiver tables
    // one tiling per kernel class (forward, adjoint, Born), picked by the
    // autotuner or forced by fwi_ctx_set_tiling
    Tiling tile[kClasses];
    int force_cw[kClasses] = {}, force_rows[kClasses] = {}, force_tb[kClasses] = {}, force_pd[kClasses] = {};
    bool autotune = true;
    // scratch
    DevBuf fields, samples, image, dhist, ckpt, partials, misfit, check, pairdata;
    DevBuf resid;   // combined off-grid receiver traces / residuals [data]
    // perfectly matched layer: edge fields of the background / forward field,
    // of the scattered field and of the adjoint field, four field-sized
    // buffers each (x and z at two levels)
    DevBuf psi;
    // RTM image product: muted data, the migrated image before the filter,
    // and the per-trace mute table (host copies kept until the next call)
    DevBuf rtm_data, rtm_img, d_mute_off, d_mute_nt, d_mute_t0;
    std::vector<int64_t> h_mute_off;
    std::vector<int32_t> h_mute_nt;
    std::vector<float> h_mute_t0;
    // copies of the call's model and perturbation: the time loops read these,
    // never the caller's buffers, so captured loops stay valid across calls
    DevBuf model, dmodel;
    // captured time loops (replayed on the caller's stream; captured on a
    // private stream, since the legacy default stream cannot be captured)
    bool graphs = true;
    hipStream_t cap_stream = nullptr;
    std::vector<GraphEntry> graph_cache;
    uint64_t graph_tick = 0;
    float *h_check = nullptr;     // pinned [3]
    double *h_misfit = nullptr;   // pinned [1]
    // the allocation-free entry points' scratch: this device's copy of the
    // static `scratch` array (device address), and, while such a call runs,
    // the bytes carved from it so far (arena != nullptr: ensure() carves
    // instead of allocating)
    unsigned char *scratch_dev = nullptr;
    unsigned char *arena = nullptr;
    size_t arena_used = 0;
    // profiling events
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
    std::vector<std::pair<int, size_t>> ev_marks;  // (class, first event index)
};

namespace {

int set_err(fwi_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPCHK(ctx, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return set_err(ctx, FWI_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

int ensure(fwi_ctx *c, DevBuf &b, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (b.bytes >= bytes) return FWI_OK;
    if (c->arena) {
        // an allocation-free call: carve the buffer from the static scratch
        // (a buffer that grows is carved again; nothing is freed)
        const size_t off = (c->arena_used + 255) & ~size_t(255);
        if (off > kNoAllocScratchBytes || bytes > kNoAllocScratchBytes - off)
            return set_err(c, FWI_ENOMEM,
                           "the allocation-free entry points have %zu bytes of scratch; this call needs more "
                           "(at least %zu)",
                           kNoAllocScratchBytes, off + bytes);
        b.p = c->arena + off;
        b.bytes = bytes;
        c->arena_used = off + bytes;
        return FWI_OK;
    }
    if (b.p) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        HIPCHK(c, hipFree(b.p));
        b.p = nullptr;
        b.bytes = 0;
    }
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return set_err(c, FWI_ENOMEM, "device allocation of %zu bytes failed", bytes);
    }
    b.bytes = bytes;
    return FWI_OK;
}

void release(DevBuf &b)
{
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

// Device address of this device's copy of `scratch` (the device must be
// current), looked up once per device.
int scratch_address(int device, unsigned char **out)
{
    static std::mutex mu;
    static std::map<int, unsigned char *> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(device);
    if (it == addr.end()) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return FWI_EHIP;
        }
        it = addr.emplace(device, static_cast<unsigned char *>(p)).first;
    }
    *out = it->second;
    return FWI_OK;
}

}  // namespace

void Tiling::release_all()
{
    for (DevBuf *b : {&d_waves, &d_rrows, &d_rmap, &d_waves1, &d_rrows1, &d_rmap1}) release(*b);
}

namespace {

void clear_graphs(fwi_ctx *c)
{
    for (GraphEntry &e : c->graph_cache)
        if (e.exec) (void)hipGraphExecDestroy(e.exec);
    c->graph_cache.clear();
}

template <class T>
int upload(fwi_ctx *c, DevBuf &b, const std::vector<T> &v)
{
    int rc = ensure(c, b, v.size() * sizeof(T));
    if (rc) return rc;
    if (!v.empty())
        HIPCHK(c, hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
    return FWI_OK;
}

template <class T>
void put(std::vector<char> &k, const T *p, size_t n)
{
    const char *b = reinterpret_cast<const char *>(p);
    k.insert(k.end(), b, b + n * sizeof(T));
}

// ---------------------------------------------------------------------------
// argument checks and the plan

int build_plan(fwi_ctx *c, const fwi_grid *g, const fwi_geom *geo)
{
    if (!g || !geo) return set_err(c, FWI_EINVAL, "grid and geometry must not be NULL");
    if (g->nz < 1 || g->nx < 1 || g->nb < 0 || g->nt_max < 1)
        return set_err(c, FWI_EINVAL, "bad grid sizes nz=%d nx=%d nb=%d nt_max=%d", g->nz, g->nx, g->nb,
                       g->nt_max);
    if (!(g->h > 0.f) || !(g->dt > 0.f) || !(g->v_ref > 0.f) || !(g->R > 0.f && g->R < 1.f))
        return set_err(c, FWI_EINVAL, "bad grid constants h=%g dt=%g v_ref=%g R=%g", g->h, g->dt, g->v_ref, g->R);
    if (double(g->v_ref) * g->dt / g->h > kCflLimit)
        return set_err(c, FWI_ECFL, "v_ref*dt/h = %.4f exceeds %.2f", double(g->v_ref) * g->dt / g->h,
                       kCflLimit);
    if (g->ckpt_every < 0) return set_err(c, FWI_EINVAL, "ckpt_every must be >= 0");
    if (g->free_surface != 0 && g->free_surface != 1) return set_err(c, FWI_EINVAL, "free_surface must be 0 or 1");
    if (g->relative != 0 && g->relative != 1) return set_err(c, FWI_EINVAL, "relative must be 0 or 1");
    if (g->pml != 0 && g->pml != 1) return set_err(c, FWI_EINVAL, "pml must be 0 or 1");
    const int top = g->free_surface ? 0 : g->nb;
    const int64_t NZ64 = int64_t(g->nz) + int64_t(g->nb) + top;
    if (NZ64 > (1 << 20) || int64_t(g->nx) + 2 * g->nb > (1 << 20))
        return set_err(c, FWI_EINVAL, "grid too large");
    const int S = geo->nshots;
    if (S < 0) return set_err(c, FWI_EINVAL, "nshots < 0");
    if (S > 0 && (!geo->src_z || !geo->src_x || !geo->rec_ptr || !geo->wavelet))
        return set_err(c, FWI_EINVAL, "NULL geometry array");
    if ((geo->win_x0 == nullptr) != (geo->win_nx == nullptr))
        return set_err(c, FWI_EINVAL, "win_x0 and win_nx must both be given or both be NULL");
    if (S > 0 && geo->rec_ptr[0] != 0) return set_err(c, FWI_EINVAL, "rec_ptr[0] must be 0");
    for (int s = 0; s < S; ++s)
        if (geo->rec_ptr[s + 1] < geo->rec_ptr[s]) return set_err(c, FWI_EINVAL, "rec_ptr not monotone");
    const int64_t nrec_tot = S > 0 ? geo->rec_ptr[S] : 0;
    if (nrec_tot > 0 && (!geo->rec_z || !geo->rec_x)) return set_err(c, FWI_EINVAL, "NULL receiver arrays");
    if (nrec_tot > (int64_t(1) << 30)) return set_err(c, FWI_EINVAL, "too many receivers");
    if ((geo->src_fz == nullptr) != (geo->src_fx == nullptr) || (geo->rec_fz == nullptr) != (geo->rec_fx == nullptr))
        return set_err(c, FWI_EINVAL, "off-grid offsets come in (fz, fx) pairs: both or neither");
    auto bad_frac = [](float f) { return !(f >= 0.f && f < 1.f); };

    // plan cache key: every input the plan depends on
    std::vector<char> key;
    put(key, g, 1);
    put(key, &S, 1);
    if (S > 0) {
        put(key, geo->src_z, S);
        put(key, geo->src_x, S);
        const int flags[3] = {geo->win_x0 != nullptr, geo->nt != nullptr, geo->wavelet_shared != 0};
        put(key, flags, 3);
        if (geo->win_x0) {
            put(key, geo->win_x0, S);
            put(key, geo->win_nx, S);
        }
        if (geo->nt) put(key, geo->nt, S);
        const int fflags[2] = {geo->src_fz != nullptr, geo->rec_fz != nullptr};
        put(key, fflags, 2);
        if (geo->src_fz) {
            put(key, geo->src_fz, S);
            put(key, geo->src_fx, S);
        }
        if (geo->rec_fz) {
            put(key, geo->rec_fz, nrec_tot);
            put(key, geo->rec_fx, nrec_tot);
        }
        put(key, geo->rec_ptr, S + 1);
        put(key, geo->rec_z, nrec_tot);
        put(key, geo->rec_x, nrec_tot);
        put(key, geo->wavelet, size_t(geo->wavelet_shared ? 1 : S) * g->nt_max);
    }
    if (c->plan_valid && key == c->plan.key) return FWI_OK;
    c->plan_valid = false;
    clear_graphs(c);

    Plan p;
    p.nz = g->nz;
    p.nx = g->nx;
    p.nb = g->nb;
    p.NZ = int(NZ64);
    p.top = top;
    p.free_surface = g->free_surface != 0;
    p.pml = g->pml != 0 && g->nb > 0;
    p.relative = g->relative != 0;
    p.nt_max = g->nt_max;
    p.h = g->h;
    p.dt = g->dt;
    p.v_ref = g->v_ref;
    p.R = g->R;
    p.ckpt_every = g->ckpt_every;
    p.S = S;

    std::vector<int> x0(S), wnx(S), nts(S);
    std::vector<int64_t> data_off(S + 1, 0);
    for (int s = 0; s < S; ++s) {
        x0[s] = geo->win_x0 ? geo->win_x0[s] : 0;
        wnx[s] = geo->win_x0 ? geo->win_nx[s] : g->nx;
        nts[s] = geo->nt ? geo->nt[s] : g->nt_max;
        if (x0[s] < 0 || wnx[s] < 1 || int64_t(x0[s]) + wnx[s] > g->nx)
            return set_err(c, FWI_EINVAL, "shot %d: window [%d, %d) outside [0, %d)", s, x0[s], x0[s] + wnx[s],
                           g->nx);
        if (nts[s] < 0 || nts[s] > g->nt_max)
            return set_err(c, FWI_EINVAL, "shot %d: nt=%d outside [0, nt_max=%d]", s, nts[s], g->nt_max);
        const int sz = geo->src_z[s], sx = geo->src_x[s];
        const float sfz = geo->src_fz ? geo->src_fz[s] : 0.f, sfx = geo->src_fz ? geo->src_fx[s] : 0.f;
        if (sz < 0 || sz >= g->nz || sx < x0[s] || sx >= x0[s] + wnx[s])
            return set_err(c, FWI_EINVAL, "shot %d: source (%d, %d) outside its window", s, sz, sx);
        if (bad_frac(sfz) || bad_frac(sfx) || (sfz > 0.f && sz + 1 >= g->nz) || (sfx > 0.f && sx + 1 >= x0[s] + wnx[s]))
            return set_err(c, FWI_EINVAL, "shot %d: source offsets (%g, %g) outside [0, 1) or the window", s,
                           double(sfz), double(sfx));
        for (int64_t r = geo->rec_ptr[s]; r < geo->rec_ptr[s + 1]; ++r) {
            const int rz = geo->rec_z[r], rx = geo->rec_x[r];
            if (rz < 0 || rz >= g->nz || rx < x0[s] || rx >= x0[s] + wnx[s])
                return set_err(c, FWI_EINVAL, "shot %d: receiver %lld at (%d, %d) outside its window", s,
                               (long long)r, rz, rx);
            const float fz = geo->rec_fz ? geo->rec_fz[r] : 0.f, fx = geo->rec_fz ? geo->rec_fx[r] : 0.f;
            if (bad_frac(fz) || bad_frac(fx) || (fz > 0.f && rz + 1 >= g->nz) || (fx > 0.f && rx + 1 >= x0[s] + wnx[s]))
                return set_err(c, FWI_EINVAL, "shot %d: receiver %lld offsets (%g, %g) outside [0, 1) or the window",
                               s, (long long)r, double(fz), double(fx));
        }
        data_off[s + 1] = data_off[s] + (geo->rec_ptr[s + 1] - geo->rec_ptr[s]) * int64_t(nts[s]);
    }
    p.data_size = data_off[S];

    // slots: record length decreasing (stable)
    p.order.resize(S);
    for (int s = 0; s < S; ++s) p.order[s] = s;
    std::stable_sort(p.order.begin(), p.order.end(), [&](int a, int b) { return nts[a] > nts[b]; });

    p.shots.resize(S);
    p.slot_nt.resize(S);
    p.slot_cells.resize(S);
    int64_t foff = 0, goff = 0;
    p.q_rptr.push_back(0);
    if (geo->wavelet_shared) p.wav.assign(geo->wavelet, geo->wavelet + g->nt_max);
    else p.wav.resize(size_t(S) * g->nt_max);
    for (int k = 0; k < S; ++k) {
        const int s = p.order[k];
        ShotDesc &d = p.shots[k];
        d.NX = wnx[s] + 2 * p.nb;
        d.P = ((d.NX + kZeroRows + 31) / 32) * 32;
        d.f_off = foff + int64_t(kRowsAbove) * d.P;
        d.g_off = goff;
        foff += int64_t(p.NZ + kRowsExtra) * d.P;
        goff += int64_t(p.NZ) * d.P;
        d.x0 = x0[s];
        d.wnx = wnx[s];
        d.nt = nts[s];
        d.src_i = geo->src_z[s] + p.top;
        d.src_j = geo->src_x[s] - x0[s] + p.nb;
        if (geo->wavelet_shared) d.wav_off = 0;
        else {
            d.wav_off = k * g->nt_max;
            std::memcpy(&p.wav[size_t(k) * g->nt_max], geo->wavelet + size_t(s) * g->nt_max,
                        sizeof(float) * g->nt_max);
        }
        p.slot_nt[k] = nts[s];
        p.updates_per_field_pass += double(p.NZ) * d.NX * nts[s];
        // bilinear weights: (1-fz)(1-fx), (1-fz)fx, fz(1-fx), fz fx
        auto weights = [](double fz, double fx, float *w) {
            w[0] = float((1.0 - fz) * (1.0 - fx));
            w[1] = float((1.0 - fz) * fx);
            w[2] = float(fz * (1.0 - fx));
            w[3] = float(fz * fx);
        };
        {
            float w[4];
            weights(geo->src_fz ? geo->src_fz[s] : 0.0, geo->src_fz ? geo->src_fx[s] : 0.0, w);
            d.sw00 = w[0];
            d.sw01 = w[1];
            d.sw10 = w[2];
            d.sw11 = w[3];
        }

        // unique receiver cells of this shot, sorted by (row, col); a
        // receiver off the grid touches the cells of its nonzero weights
        std::map<std::pair<int, int>, std::vector<std::pair<int64_t, float>>> cells;
        std::vector<std::vector<std::pair<std::pair<int, int>, float>>> rec_cells;
        for (int64_t r = geo->rec_ptr[s]; r < geo->rec_ptr[s + 1]; ++r) {
            const int i = geo->rec_z[r] + p.top, jj = geo->rec_x[r] - x0[s] + p.nb;
            const int64_t off = data_off[s] + (r - geo->rec_ptr[s]) * int64_t(nts[s]);
            float w[4];
            weights(geo->rec_fz ? geo->rec_fz[r] : 0.0, geo->rec_fz ? geo->rec_fx[r] : 0.0, w);
            rec_cells.emplace_back();
            for (int ab = 0; ab < 4; ++ab) {
                if (w[ab] == 0.f) continue;
                const std::pair<int, int> cell{i + ab / 2, jj + ab % 2};
                cells[cell].push_back({off, w[ab]});
                rec_cells.back().push_back({cell, w[ab]});
                if (w[ab] != 1.f) p.offgrid = true;
            }
            p.r_off.push_back(off);
            p.r_nt.push_back(nts[s]);
        }
        std::map<std::pair<int, int>, int> qof;
        for (auto &kv : cells) {
            p.slot_cells[k].push_back({kv.first, p.Q});
            qof[kv.first] = p.Q;
            p.q_nt.push_back(nts[s]);
            for (auto &ow : kv.second) {
                p.q_roff.push_back(ow.first);
                p.q_rw.push_back(ow.second);
            }
            p.q_rptr.push_back(int32_t(p.q_roff.size()));
            ++p.Q;
        }
        for (auto &rc : rec_cells) {
            if (p.r_cptr.empty()) p.r_cptr.push_back(0);
            for (auto &cw : rc) {
                p.r_cq.push_back(qof[cw.first]);
                p.r_cw.push_back(cw.second);
            }
            p.r_cptr.push_back(int32_t(p.r_cq.size()));
            ++p.nrec;
        }
    }
    p.field_floats = foff;
    p.img_floats = goff;
    for (int k = 0; k < S; ++k)
        if (int64_t(p.NZ + kRowsExtra) * p.shots[k].P >= (int64_t(1) << 31))
            return set_err(c, FWI_EINVAL, "shot %d: padded field too large", k);
    p.key = std::move(key);

    int rc;
    if ((rc = upload(c, c->d_shots, p.shots)) || (rc = upload(c, c->d_qnt, p.q_nt)) || (rc = upload(c, c->d_qrptr, p.q_rptr)) ||
        (rc = upload(c, c->d_qroff, p.q_roff)) || (rc = upload(c, c->d_wav, p.wav)))
        return rc;
    if (p.offgrid) {
        if ((rc = upload(c, c->d_qrw, p.q_rw)) || (rc = upload(c, c->d_rcptr, p.r_cptr)) ||
            (rc = upload(c, c->d_rcq, p.r_cq)) || (rc = upload(c, c->d_rnt, p.r_nt)) ||
            (rc = upload(c, c->d_rcw, p.r_cw)) || (rc = upload(c, c->d_roff, p.r_off)) ||
            (rc = ensure(c, c->resid, size_t(std::max<int64_t>(p.data_size, 1)) * 4)))
            return rc;
    }
    // the host vectors are read by the copies above; keep them alive in the
    // context and make sure the copies finished before the plan can change
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->plan = std::move(p);
    for (Tiling &t : c->tile) t.cw = t.rows = t.tb = 0;  // stale for the new plan
    c->plan_valid = true;
    return FWI_OK;
}

// Wave table of one tiling. One level per launch: a wave owns a strip of
// 64*cw columns; two levels per launch: a strip of 64*cw - 8 columns whose
// lanes also hold 4 columns on each side, and the receiver maps cover the
// lanes' columns and 4 rows above and below the owned rows (the
// intermediate level is computed there too).
void build_tiling(const Plan &p, int cw, int rows_target, int tb, int pd, Tiling &t)
{
    t.cw = cw;
    t.rows = rows_target;
    t.tb = tb;
    t.pd = pd;
    t.waves.clear();
    t.rrows.clear();
    t.rmap.clear();
    t.prefix.assign(p.S + 1, 0);
    const int SW = kLanes * cw;
    const int reach = tb == 2 ? kHalo : 0;
    const int SWo = SW - 2 * reach;
    const int nseg = std::max(1, (p.NZ + rows_target - 1) / rows_target);
    const int rows = (p.NZ + nseg - 1) / nseg;
    for (int k = 0; k < p.S; ++k) {
        const auto &cells = p.slot_cells[k];
        const int nstrips = (p.shots[k].NX + SWo - 1) / SWo;
        // receiver cells of each strip, sorted by row, then column
        std::vector<std::vector<std::pair<std::pair<int, int>, int>>> strip_cells(nstrips);
        for (int st = 0; st < nstrips; ++st) {
            const int lane0 = st * SWo - reach;
            for (const auto &cq : cells)
                if (cq.first.second >= lane0 && cq.first.second < lane0 + SW) strip_cells[st].push_back(cq);
        }
        // adjacent strips of one row band get consecutive wave ids: the waves
        // of a workgroup start together and read neighbouring stretches of
        // each row at about the same time
        for (int z0 = 0; z0 < p.NZ; z0 += rows) {
            for (int st = 0; st < nstrips; ++st) {
                const int col0 = st * SWo, lane0 = col0 - reach;
                const auto &sc = strip_cells[st];
                WaveDesc w{};
                w.shot = k;
                w.col0 = col0;
                w.z0 = z0;
                w.z1 = std::min(p.NZ, z0 + rows);
                w.rr0 = int(t.rrows.size());
                const int rlo = w.z0 - reach, rhi = w.z1 + reach;
                size_t pos = 0;
                while (pos < sc.size() && sc[pos].first.first < rlo) ++pos;
                while (pos < sc.size() && sc[pos].first.first < rhi) {
                    const int rowi = sc[pos].first.first;
                    RecRow rrw{rowi, int32_t(t.rmap.size())};
                    t.rmap.resize(t.rmap.size() + SW, -1);
                    while (pos < sc.size() && sc[pos].first.first == rowi) {
                        t.rmap[rrw.map_off + (sc[pos].first.second - lane0)] = sc[pos].second;
                        ++pos;
                    }
                    t.rrows.push_back(rrw);
                }
                w.rr1 = int(t.rrows.size());
                t.waves.push_back(w);
            }
        }
        t.prefix[k + 1] = int(t.waves.size());
    }
    t.waves1.clear();
    t.rrows1.clear();
    t.rmap1.clear();
    t.prefix1.clear();
    if (tb == 2) {
        Tiling one;
        build_tiling(p, cw, rows_target, 1, 1, one);
        t.waves1 = std::move(one.waves);
        t.rrows1 = std::move(one.rrows);
        t.rmap1 = std::move(one.rmap);
        t.prefix1 = std::move(one.prefix);
    }
}

int upload_tiling(fwi_ctx *c, Tiling &t)
{
    int rc;
    if ((rc = upload(c, t.d_waves, t.waves)) || (rc = upload(c, t.d_rrows, t.rrows)) ||
        (rc = upload(c, t.d_rmap, t.rmap)))
        return rc;
    if (t.tb == 2 && ((rc = upload(c, t.d_waves1, t.waves1)) || (rc = upload(c, t.d_rrows1, t.rrows1)) ||
                      (rc = upload(c, t.d_rmap1, t.rmap1))))
        return rc;
    // pageable sources: make sure the copies have consumed them
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return FWI_OK;
}

// copy of a caller's [nz][nx] array into a context buffer (enqueued)
int copy_in(fwi_ctx *c, const float *src, DevBuf &dst, const float **out)
{
    const Plan &p = c->plan;
    const size_t bytes = size_t(p.nz) * p.nx * sizeof(float);
    int rc = ensure(c, dst, bytes);
    if (rc) return rc;
    HIPCHK(c, hipMemcpyAsync(dst.p, src, bytes, hipMemcpyDeviceToDevice, c->stream));
    *out = static_cast<const float *>(dst.p);
    return FWI_OK;
}

// Validates the model and copies it into the context; *out is the copy,
// which every later step of the call reads.
int check_model(fwi_ctx *c, const float *&v, const char *what)
{
    const Plan &p = c->plan;
    if (!v) return set_err(c, FWI_EINVAL, "%s is NULL", what);
    int rc = ensure(c, c->check, 4 * sizeof(float));
    if (rc) return rc;
    HIPCHK(c, launch_model_check(v, int64_t(p.nz) * p.nx, static_cast<float *>(c->check.p), c->stream));
    HIPCHK(c, hipMemcpyAsync(c->h_check, c->check.p, 3 * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->h_check[2] > 0.f)
        return set_err(c, FWI_EINVAL, "%s has %.0f non-finite or non-positive entries", what, c->h_check[2]);
    const double cfl = double(c->h_check[1]) * p.dt / p.h;
    if (cfl > kCflLimit)
        return set_err(c, FWI_ECFL, "max(%s)*dt/h = %.4f exceeds %.2f", what, cfl, kCflLimit);
    return copy_in(c, v, c->model, &v);
}

// The perturbation may take any sign; it is copied into the context.
int check_perturbation(fwi_ctx *c, const float *&dv)
{
    if (!dv) return set_err(c, FWI_EINVAL, "dv is NULL");
    return copy_in(c, dv, c->dmodel, &dv);
}

StepArgs base_args(fwi_ctx *c, const float *v, int cls)
{
    const Plan &p = c->plan;
    const Tiling &t = c->tile[cls];
    StepArgs a{};
    a.shots = static_cast<const ShotDesc *>(c->d_shots.p);
    a.waves = static_cast<const WaveDesc *>(t.d_waves.p);
    a.rrows = static_cast<const RecRow *>(t.d_rrows.p);
    a.rmap = static_cast<const int32_t *>(t.d_rmap.p);
    a.cw = t.cw;
    a.pd = t.pd;
    a.v = v;
    a.wav = static_cast<const float *>(c->d_wav.p);
    a.nz = p.nz;
    a.nx = p.nx;
    a.nb = p.nb;
    a.top = p.top;
    a.fs = p.free_surface ? 1 : 0;
    a.rel = p.relative ? 1 : 0;
    a.NZ = p.NZ;
    const double ih2 = 1.0 / (double(p.h) * p.h);
    a.w1 = float(kC8[1] * ih2);
    a.w2 = float(kC8[2] * ih2);
    a.w3 = float(kC8[3] * ih2);
    a.w4 = float(kC8[4] * ih2);
    a.dt2 = float(double(p.dt) * p.dt);
    a.ih2 = float(ih2);
    if (p.nb > 0) {
        const double smax = 3.0 * p.v_ref * std::log(1.0 / p.R) / (2.0 * p.nb * p.h);
        a.hs = float(smax * p.dt / (2.0 * double(p.nb) * p.nb));
        a.hd0 = float(smax / (4.0 * double(p.nb) * p.nb));
    }
    a.pml = p.pml ? 1 : 0;
    a.dt = p.dt;
    a.ih = float(1.0 / double(p.h));
    return a;
}

// ---- profiling --------------------------------------------------------------

int ev_begin(fwi_ctx *c, int cls)
{
    if (!c->profiling) return FWI_OK;
    if (c->ev_used + 2 > c->ev.size()) {
        const size_t add = std::max<size_t>(256, c->ev.size());
        for (size_t i = 0; i < add; ++i) {
            hipEvent_t e;
            HIPCHK(c, hipEventCreate(&e));
            c->ev.push_back(e);
        }
    }
    c->ev_marks.push_back({cls, c->ev_used});
    HIPCHK(c, hipEventRecord(c->ev[c->ev_used], c->stream));
    c->ev_used += 2;
    return FWI_OK;
}

int ev_end(fwi_ctx *c)
{
    if (!c->profiling) return FWI_OK;
    HIPCHK(c, hipEventRecord(c->ev[c->ev_marks.back().second + 1], c->stream));
    return FWI_OK;
}

int ev_collect(fwi_ctx *c)
{
    if (!c->profiling) return FWI_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto &m : c->ev_marks) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev[m.second], c->ev[m.second + 1]));
        switch (m.first) {
        case K_FWD: c->stats.ms_fwd += ms; break;
        case K_ADJ: c->stats.ms_adj += ms; break;
        case K_BORN: c->stats.ms_born += ms; break;
        default: c->stats.ms_other += ms; break;
        }
    }
    c->ev_marks.clear();
    c->ev_used = 0;
    return FWI_OK;
}

// ---- sweeps -------------------------------------------------------------------

// Algorithmic bytes per cell-update: forward reads u^n, u^{n-1} and the
// model and writes u^{n+1} (16 B); emitting D^n adds a 4 B write; the
// adjoint with imaging adds the D^n read and the G read-modify-write (28 B);
// the Born step moves 32 B for its two field updates.
constexpr double kBytesFwd = 16.0, kBytesEmit = 4.0, kBytesAdj = 28.0, kBytesBorn = 32.0;
// scattered field from the stored history: du^n, du^{n-1}, v, dv, D^n in, du^{n+1} out
constexpr double kBytesScat = 24.0;

double step_updates(const Plan &p, int n)
{
    double u = 0;
    for (int k = 0; k < p.S && p.slot_nt[k] > n; ++k) u += double(p.NZ) * p.shots[k].NX;
    return u;
}

double bytes_per_update(int flags)
{
    if (flags & F_IMAGE) return kBytesAdj;
    return kBytesFwd + ((flags & F_EMIT) ? kBytesEmit : 0.0);
}

// Algorithmic bytes per cell of a two-level launch (both levels): the
// fields of levels n and n-1 and the model in, levels n+1 and n+2 out (20 B);
// each level's D adds 4 B (written, or read by the adjoint), and the image
// is read and written once for both levels.
double bytes_two_levels(int flags)
{
    if (flags & F_IMAGE) return 20.0 + 2 * kBytesEmit + 8.0;
    if (flags & F_SCAT) return 20.0 + 2 * kBytesEmit + 4.0;   // D^n, D^{n+1} and dV in
    return 20.0 + ((flags & F_EMIT) ? 2 * kBytesEmit : 0.0);
}

// ---- captured time loops -----------------------------------------------------

// the counters a time loop adds to the statistics
fwi_stats loop_delta(const fwi_stats &after, const fwi_stats &before)
{
    fwi_stats d{};
    d.cell_updates = after.cell_updates - before.cell_updates;
    d.stencil_launches = after.stencil_launches - before.stencil_launches;
    d.n_fwd = after.n_fwd - before.n_fwd;
    d.n_adj = after.n_adj - before.n_adj;
    d.n_born = after.n_born - before.n_born;
    d.bytes_fwd = after.bytes_fwd - before.bytes_fwd;
    d.bytes_adj = after.bytes_adj - before.bytes_adj;
    d.bytes_born = after.bytes_born - before.bytes_born;
    return d;
}

void loop_add(fwi_stats &s, const fwi_stats &d)
{
    s.cell_updates += d.cell_updates;
    s.stencil_launches += d.stencil_launches;
    s.n_fwd += d.n_fwd;
    s.n_adj += d.n_adj;
    s.n_born += d.n_born;
    s.bytes_fwd += d.bytes_fwd;
    s.bytes_adj += d.bytes_adj;
    s.bytes_born += d.bytes_born;
}

// Runs a time loop: `body(f)` enqueues its launches on c->stream and rotates
// `f`. With graphs on, the first run with a given key is captured on the
// private stream, instantiated and launched on the caller's stream; later
// runs with the same key replay the graph. Keys hold every pointer and
// scalar the launches take, and the cache is cleared whenever the plan or a
// tiling is rebuilt, so a replay launches exactly what the body would.
template <class Body>
int run_loop(fwi_ctx *c, const std::vector<char> &key, Fields &f, Body &&body)
{
    if (!c->graphs) return body(f);
    for (GraphEntry &e : c->graph_cache)
        if (e.key == key) {
            HIPCHK(c, hipGraphLaunch(e.exec, c->stream));
            loop_add(c->stats, e.delta);
            c->stats.graph_launches += 1;
            f = e.after;
            e.used = ++c->graph_tick;
            return FWI_OK;
        }
    if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    const fwi_stats before = c->stats;
    hipStream_t user = c->stream;
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    c->stream = c->cap_stream;
    int rc = body(f);
    c->stream = user;
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(c->cap_stream, &graph);
    if (rc || ec != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        if (rc) return rc;
        return set_err(c, FWI_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(ec));
    }
    size_t nodes = 0;
    if (hipGraphGetNodes(graph, nullptr, &nodes) == hipSuccess && nodes == 0) {
        (void)hipGraphDestroy(graph);   // nothing to run (no active shots)
        return FWI_OK;
    }
    GraphEntry e;
    e.key = key;
    e.nodes = nodes;
    const hipError_t ei = hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return set_err(c, FWI_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
    const hipError_t el = hipGraphLaunch(e.exec, c->stream);
    if (el != hipSuccess) {
        (void)hipGraphExecDestroy(e.exec);
        return set_err(c, FWI_EHIP, "hipGraphLaunch: %s", hipGetErrorString(el));
    }
    e.delta = loop_delta(c->stats, before);
    e.after = f;
    e.used = ++c->graph_tick;
    c->stats.graph_captures += 1;
    c->stats.graph_launches += 1;
    c->graph_cache.push_back(std::move(e));
    // least recently used entries go first; a destroyed graph's launches stay
    // ordered before anything enqueued later
    size_t total = 0;
    for (const GraphEntry &g : c->graph_cache) total += g.nodes;
    while (total > kGraphNodeBudget && c->graph_cache.size() > 1) {
        size_t lru = 0;
        for (size_t i = 1; i < c->graph_cache.size(); ++i)
            if (c->graph_cache[i].used < c->graph_cache[lru].used) lru = i;
        total -= c->graph_cache[lru].nodes;
        (void)hipGraphExecDestroy(c->graph_cache[lru].exec);
        c->graph_cache.erase(c->graph_cache.begin() + lru);
    }
    return FWI_OK;
}

template <class T>
void key_put(std::vector<char> &k, const T &x)
{
    const char *b = reinterpret_cast<const char *>(&x);
    k.insert(k.end(), b, b + sizeof(T));
}

// One launch of the forward or adjoint step kernel advancing `levels` (1 or
// 2) time levels; a.n / a.n2 and the per-level pointers are set by the
// caller. `active_n` selects the shots that take part (record length >
// active_n).
int step_launch(fwi_ctx *c, StepArgs a, int cls, int flags, int levels, int active_n, Fields &f)
{
    const Plan &p = c->plan;
    const Tiling &t = c->tile[cls];
    a.nwaves = t.prefix[p.active_slots(active_n)];
    a.cur = f.cur;
    a.prev = f.prev;
    a.psx_in = f.px;
    a.psz_in = f.pz;
    a.psx_out = f.qx;
    a.psz_out = f.qz;
    if (levels == 1 && t.tb == 2) {
        // the single step of a two-level tiling runs on its one-level table
        a.waves = static_cast<const WaveDesc *>(t.d_waves1.p);
        a.rrows = static_cast<const RecRow *>(t.d_rrows1.p);
        a.rmap = static_cast<const int32_t *>(t.d_rmap1.p);
        a.nwaves = t.prefix1[p.active_slots(active_n)];
        a.pd = 1;
    }
    if (levels == 2) {
        a.out1 = f.s0;
        a.out2 = f.s1;
        HIPCHK(c, launch_step2(flags, a, c->stream));
        f = Fields{f.s0, f.s1, f.prev, f.cur, f.qx, f.qz, f.px, f.pz};
    } else {
        HIPCHK(c, launch_step(flags, a, c->stream));
        std::swap(f.prev, f.cur);
        std::swap(f.px, f.qx);
        std::swap(f.pz, f.qz);
    }
    const double cells = step_updates(p, active_n);
    const double upd = levels * cells;
    const double bytes = levels == 2 ? cells * bytes_two_levels(flags)
                                     : cells * (cls == K_SCAT ? kBytesScat : bytes_per_update(flags));
    c->stats.cell_updates += upd;
    c->stats.stencil_launches += 1;
    if (cls == K_SCAT) {
        c->stats.n_born += 1;
        c->stats.bytes_born += bytes;
    } else if (cls == K_ADJ) {
        c->stats.n_adj += 1;
        c->stats.bytes_adj += bytes;
    } else {
        c->stats.n_fwd += 1;
        c->stats.bytes_fwd += bytes;
    }
    return FWI_OK;
}

// Forward steps lo .. hi-1 (pairs when the tiling runs two levels). D^n goes
// to slot n - dlo of `dh` (when emit), samples to samp + n*Q (when sample).
int forward_range_direct(fwi_ctx *c, StepArgs a, int lo, int hi, bool sample, float *samp, bool emit, float *dh,
                         int dlo, Fields &f)
{
    const Plan &p = c->plan;
    const int64_t gf = p.img_floats;
    const int flags = F_SRC | (sample ? F_SAMPLE : 0) | (emit ? F_EMIT : 0);
    const bool two = c->tile[K_FWD].tb == 2;
    int rc;
    for (int n = lo; n < hi;) {
        const int levels = (two && n + 1 < hi) ? 2 : 1;
        a.n = n;
        a.n2 = n + 1;
        if (sample) {
            a.samp = samp + size_t(n) * p.Q;
            a.samp2 = samp + size_t(n + 1) * p.Q;
        }
        if (emit) {
            a.dslot = dh + size_t(n - dlo) * gf;
            a.dslot2 = dh + size_t(n + 1 - dlo) * gf;
        }
        if ((rc = step_launch(c, a, K_FWD, flags, levels, n, f))) return rc;
        n += levels;
    }
    return FWI_OK;
}

int forward_range(fwi_ctx *c, const StepArgs &a, int lo, int hi, bool sample, float *samp, bool emit, float *dh,
                  int dlo, Fields &f)
{
    if (lo >= hi) return FWI_OK;
    std::vector<char> key;
    key_put(key, 'F');
    key_put(key, a);
    key_put(key, lo);
    key_put(key, hi);
    key_put(key, sample);
    key_put(key, samp);
    key_put(key, emit);
    key_put(key, dh);
    key_put(key, dlo);
    key_put(key, f);
    return run_loop(c, key, f, [&](Fields &ff) {
        return forward_range_direct(c, a, lo, hi, sample, samp, emit, dh, dlo, ff);
    });
}

int other(fwi_ctx *c, hipError_t e, const char *what)
{
    if (e != hipSuccess) return set_err(c, FWI_EHIP, "%s: %s", what, hipGetErrorString(e));
    return FWI_OK;
}

// ---- perfectly matched layer: edge-field buffers ------------------------------
// Block PSI_FWD holds the forward (or background) field's edge fields, PSI_SCAT
// the scattered field's, PSI_ADJ the adjoint field's: x and z at the previous
// level, then x and z at the next. Outside the layer's rows and strips they
// stay zero (the kernels never write there), so a block is zeroed once per
// sweep.
enum PsiBlock { PSI_FWD = 0, PSI_SCAT = 1, PSI_ADJ = 2 };
constexpr int kPsiBlocks = 3;

int ensure_psi(fwi_ctx *c)
{
    const Plan &p = c->plan;
    if (!p.pml) return FWI_OK;
    return ensure(c, c->psi, size_t(4 * kPsiBlocks) * size_t(p.field_floats) * 4);
}

float *psi_block(fwi_ctx *c, int b)
{
    if (!c->plan.pml) return nullptr;
    return static_cast<float *>(c->psi.p) + size_t(4 * b) * size_t(c->plan.field_floats);
}

int zero_psi(fwi_ctx *c, int b)
{
    if (!c->plan.pml) return FWI_OK;
    return other(c, launch_fill(psi_block(c, b), 4 * c->plan.field_floats, 0.f, c->stream), "fill");
}

Fields with_psi(Fields f, float *P, int64_t ff)
{
    if (P) {
        f.px = P;
        f.pz = P + ff;
        f.qx = P + 2 * ff;
        f.qz = P + 3 * ff;
    }
    return f;
}

// fields per snapshot of a forward state: (u^{n-1}, u^n) and, with the
// layer, the edge fields of level n-1
int snap_fields(const Plan &p) { return p.pml ? 4 : 2; }

void reset_stats(fwi_ctx *c)
{
    c->stats = fwi_stats{};
}

int finish_stats(fwi_ctx *c)
{
    c->stats.scratch_bytes = int64_t(c->fields.bytes + c->samples.bytes + c->image.bytes + c->dhist.bytes +
                                     c->ckpt.bytes + c->partials.bytes);
    return ev_collect(c);
}

// Checkpointing of the adjoint sweeps. The time axis is cut into segments
// of k steps. Going backward, segment by segment from the last, the adjoint
// needs that segment's D^n history, recomputed into a k-slot buffer from the
// state (u^{lo-1}, u^lo) at the segment's start. Those states come from S
// snapshot slots placed by the binomial rule of Griewank's revolve
// (Griewank & Walther, ACM TOMS 26, 2000): with s snapshots (the zero state
// at segment 0 counts as one) and at most r recomputations of any segment,
// beta(s, r) = C(s + r, s) segments can be reversed; for l segments, with r
// the least such that beta(s, r) >= l, placing the next snapshot after
// max(beta(s, r - 2), l - beta(s - 1, r)) segments reverses them with the
// fewest recomputed segments, r l - C(s + r, s + 1) in all. The forward
// sweep that computes the data passes every segment once: it stores the
// snapshots the first splits ask for and keeps the last segment's history,
// so with S >= nseg - 2 every segment but the last is recomputed exactly
// once (uniform checkpointing), and with fewer snapshots the sweep still
// runs, recomputing more.

// C(n, k), saturating at 2^62
int64_t binom_sat(int n, int k)
{
    if (k < 0 || n < 0 || k > n) return 0;
    k = std::min(k, n - k);
    const __int128 cap = __int128(1) << 62;
    __int128 r = 1;
    for (int i = 1; i <= k; ++i) {
        r = r * (n - k + i) / i;
        if (r >= cap) return int64_t(cap);
    }
    return int64_t(r);
}

// segments left of the next snapshot when l >= 2 segments are reversed with
// s >= 2 snapshots
int revolve_left(int l, int s)
{
    int r = 0;
    while (binom_sat(s + r, s) < l) ++r;
    const int64_t a = r >= 2 ? binom_sat(s + r - 2, s) : 1;
    const int64_t m = std::max<int64_t>(a, int64_t(l) - binom_sat(s + r - 1, s - 1));
    return int(std::min<int64_t>(std::max<int64_t>(m, 1), l - 1));
}

// segments recomputed by the backward sweep over nseg segments with `slots`
// snapshot slots (the closed form above, s = slots + 1)
int64_t revolve_recompute(int nseg, int slots)
{
    const int s = slots + 1;
    int r = 0;
    while (binom_sat(s + r, s) < nseg) ++r;
    return int64_t(r) * nseg - binom_sat(s + r, s + 1);
}

std::vector<int> revolve_free(int slots)
{
    std::vector<int> f;
    for (int q = slots - 1; q >= 0; --q) f.push_back(q);   // slot 0 is used first
    return f;
}

// snapshots the forward sweep stores: spine[sgi] = slot holding the state at
// the start of segment sgi, -1 for none
std::vector<int> revolve_spine(int nseg, int slots)
{
    std::vector<int> spine(size_t(std::max(nseg, 0)), -1), free = revolve_free(slots);
    int lo = 0, s = 1 + slots;
    while (nseg - lo > 1 && s >= 2) {
        const int m = lo + revolve_left(nseg - lo, s);
        spine[size_t(m)] = free.back();
        free.pop_back();
        lo = m;
        --s;
    }
    return spine;
}

// Reverse segments [lo, hi), the state at segment lo being in snapshot
// `root` (-1: the zero state), with the free slots `free` (taken from the
// back). On the first-split path (hi == nseg) the forward sweep has stored
// the snapshots and the last segment's history. Ops provides restore(slot,
// seg), advance(seg0, seg1), store(slot, seg), emit(seg) (recompute the
// segment storing its history) and adjoint(seg). A split reverses the part
// right of the new snapshot, frees the snapshot, then reverses the part
// left of it; the pending work is kept on an explicit stack (with ample
// snapshots the splits nest once per segment).
template <class Ops>
int revolve(Ops &op, int nseg, int lo0, int hi0, int root0, std::vector<int> &free)
{
    struct Task {
        int lo, hi, root;
        bool release;   // only return `root` to the free slots
    };
    std::vector<Task> todo{{lo0, hi0, root0, false}};
    int rc;
    while (!todo.empty()) {
        const Task t = todo.back();
        todo.pop_back();
        if (t.release) {
            free.push_back(t.root);
            continue;
        }
        const int lo = t.lo, hi = t.hi, root = t.root;
        const bool spine = hi == nseg;
        const int l = hi - lo;
        if (l == 1) {
            if (!spine && ((rc = op.restore(root, lo)) || (rc = op.emit(lo)))) return rc;
            if ((rc = op.adjoint(lo))) return rc;
            continue;
        }
        const int s = 1 + int(free.size());
        if (s == 1) {
            for (int j = hi - 1; j >= lo; --j) {
                if (!(spine && j == nseg - 1))
                    if ((rc = op.restore(root, lo)) || (rc = op.advance(lo, j)) || (rc = op.emit(j))) return rc;
                if ((rc = op.adjoint(j))) return rc;
            }
            continue;
        }
        const int m = lo + revolve_left(l, s);
        const int slot = free.back();
        free.pop_back();
        if (!spine)
            if ((rc = op.restore(root, lo)) || (rc = op.advance(lo, m)) || (rc = op.store(slot, m))) return rc;
        todo.push_back({lo, m, root, false});
        todo.push_back({0, 0, slot, true});
        todo.push_back({m, hi, slot, false});
    }
    return FWI_OK;
}

// Replays a schedule on the host, checking every action against the state
// it tracks; counts the recomputed segments.
struct RevolveCheck {
    int pos = -1;                 // segment whose start the current state is at (-1: none)
    int hist = -1;                // segment whose history is in the buffer
    int next_adj = 0;             // segment the adjoint must take next
    std::vector<int> held;        // slot -> segment start it holds (-1: none)
    int64_t forwards = 0;
    int restore(int slot, int seg)
    {
        const int at = slot < 0 ? 0 : held[size_t(slot)];
        if (at != seg) return FWI_ESTATE;
        pos = seg;
        return FWI_OK;
    }
    int advance(int a, int b)
    {
        if (pos != a || b < a) return FWI_ESTATE;
        forwards += b - a;
        pos = b;
        return FWI_OK;
    }
    int store(int slot, int seg)
    {
        if (pos != seg) return FWI_ESTATE;
        held[size_t(slot)] = seg;
        return FWI_OK;
    }
    int emit(int seg)
    {
        if (pos != seg) return FWI_ESTATE;
        forwards += 1;
        hist = seg;
        pos = seg + 1;
        return FWI_OK;
    }
    int adjoint(int seg)
    {
        if (seg != next_adj || hist != seg) return FWI_ESTATE;
        --next_adj;
        return FWI_OK;
    }
};

int revolve_check(int nseg, int slots, int64_t *forwards)
{
    if (nseg < 1 || slots < 0) return FWI_EINVAL;
    RevolveCheck ck;
    ck.held.assign(size_t(slots), -1);
    const std::vector<int> spine = revolve_spine(nseg, slots);
    for (int q = 0; q < nseg; ++q)
        if (spine[size_t(q)] >= 0) ck.held[size_t(spine[size_t(q)])] = q;
    ck.hist = nseg - 1;           // the forward sweep kept the last segment's history
    ck.next_adj = nseg - 1;
    std::vector<int> free = revolve_free(slots);
    int rc = revolve(ck, nseg, 0, nseg, -1, free);
    if (rc == FWI_OK && ck.next_adj != -1) rc = FWI_ESTATE;
    if (forwards) *forwards = ck.forwards;
    return rc;
}

struct Sweep {
    int k = 0, nseg = 0, slots = 0;
    std::vector<int> spine;       // snapshot slot stored at each segment start (-1: none)
    float *F[4], *A[4], *Dh, *CK, *G;
};

// Choose the segment length k and the snapshot slots. Memory = k history
// slots + S snapshots of (u^{n-1}, u^n). Uniform checkpointing (S = nseg - 2,
// no segment recomputed twice) at the k that fits the budget; if none does,
// the (k, S) within the budget with the fewest recomputed steps.
int choose_segments(fwi_ctx *c, Sweep &w)
{
    const Plan &p = c->plan;
    const int nt = p.nt_max;
    const double slot = double(p.img_floats) * 4.0;
    const double ck = double(snap_fields(p)) * double(p.field_floats) * 4.0;
    auto nseg_of = [&](int k) { return (nt + k - 1) / k; };
    auto uniform = [&](int k) { return std::max(0, nseg_of(k) - 2); };
    auto mem = [&](int k, int S) { return double(k) * slot + double(S) * ck; };
    int k, S;
    if (p.ckpt_every > 0) {
        k = std::min(p.ckpt_every, std::max(nt, 1));
        S = uniform(k);
    } else {
        // never plan beyond what is free now (plus what this context already
        // holds for the same purpose), keeping a margin for the caller
        size_t fr = 0, tot = 0;
        double budget = double(c->budget);
        if (hipMemGetInfo(&fr, &tot) == hipSuccess) {
            const double avail = double(fr) + double(c->dhist.bytes) + double(c->ckpt.bytes) - double(kFreeMargin);
            budget = std::min(budget, std::max(avail, 0.0));
        }
        k = std::max(nt, 1);
        S = uniform(k);
        if (mem(k, S) > budget) {
            k = int(std::max(1.0, std::min(double(nt), std::floor(budget / std::max(slot, 1.0)))));
            while (k > 1 && mem(k, uniform(k)) > budget) k = std::max(1, k - std::max(1, k / 32));
            S = uniform(k);
            if (mem(k, S) > budget) {
                // binomial: the fewest recomputed steps over all k
                double best = -1.0;
                for (int kk = 1; kk <= nt; ++kk) {
                    const double room = budget - double(kk) * slot;
                    if (room < 0.0) break;
                    const int SS = int(std::min<double>(uniform(kk), std::floor(room / std::max(ck, 1.0))));
                    const double cost = double(kk) * double(revolve_recompute(nseg_of(kk), SS));
                    if (best < 0.0 || cost < best) {
                        best = cost;
                        k = kk;
                        S = SS;
                    }
                }
                if (best < 0.0)
                    return set_err(c, FWI_ENOMEM, "memory budget %.3g B too small for the adjoint sweep", budget);
            }
        }
    }
    if (c->ckpt_slots >= 0) S = std::min(S, c->ckpt_slots);
    w.k = k;
    w.nseg = nseg_of(k);
    w.slots = S;
    w.spine = revolve_spine(w.nseg, S);
    c->stats.ckpt_every = w.nseg > 1 ? k : 0;
    c->stats.n_segments = w.nseg;
    c->stats.ckpt_slots = S;
    return FWI_OK;
}

// Forward sweep for an adjoint: the snapshots of (u^{n-1}, u^n) the
// checkpointing schedule asks for, D^n stored for the last segment, receiver
// samples (time-major) if `sample`.
int forward_for_adjoint(fwi_ctx *c, const float *v, bool sample, Sweep &w)
{
    const Plan &p = c->plan;
    int rc;
    if ((rc = choose_segments(c, w))) return rc;
    const int k = w.k, nseg = w.nseg;
    const int64_t ff = p.field_floats, gf = p.img_floats;
    const int sf = snap_fields(p);
    if ((rc = ensure(c, c->fields, size_t(8 * ff) * 4)) || (rc = ensure(c, c->image, size_t(gf) * 4)) ||
        (rc = ensure(c, c->dhist, size_t(k) * gf * 4)) ||
        (rc = ensure(c, c->ckpt, size_t(w.slots) * sf * ff * 4)) ||
        (rc = ensure(c, c->samples, size_t(p.nt_max) * p.Q * 4)) || (rc = ensure_psi(c)))
        return rc;
    float *F = static_cast<float *>(c->fields.p);
    for (int i = 0; i < 4; ++i) {
        w.F[i] = F + i * ff;
        w.A[i] = F + (4 + i) * ff;
    }
    w.Dh = static_cast<float *>(c->dhist.p);
    w.CK = static_cast<float *>(c->ckpt.p);
    w.G = static_cast<float *>(c->image.p);
    float *samp = static_cast<float *>(c->samples.p);
    hipStream_t st = c->stream;
    if ((rc = other(c, launch_fill(w.F[0], 4 * ff, 0.f, st), "fill")) || (rc = zero_psi(c, PSI_FWD))) return rc;
    StepArgs a = base_args(c, v, K_FWD);
    Fields f = with_psi(Fields{w.F[0], w.F[1], w.F[2], w.F[3]}, psi_block(c, PSI_FWD), ff);
    if ((rc = ev_begin(c, K_FWD))) return rc;
    for (int sgi = 0; sgi < nseg; ++sgi) {
        const int lo = sgi * k, hi = std::min(p.nt_max, lo + k);
        const bool last = sgi == nseg - 1;
        if (w.spine[size_t(sgi)] >= 0) {
            float *ckp = w.CK + size_t(w.spine[size_t(sgi)]) * sf * ff;
            HIPCHK(c, hipMemcpyAsync(ckp, f.prev, size_t(ff) * 4, hipMemcpyDeviceToDevice, st));
            HIPCHK(c, hipMemcpyAsync(ckp + ff, f.cur, size_t(ff) * 4, hipMemcpyDeviceToDevice, st));
            if (p.pml) {
                HIPCHK(c, hipMemcpyAsync(ckp + 2 * ff, f.px, size_t(ff) * 4, hipMemcpyDeviceToDevice, st));
                HIPCHK(c, hipMemcpyAsync(ckp + 3 * ff, f.pz, size_t(ff) * 4, hipMemcpyDeviceToDevice, st));
            }
        }
        if ((rc = forward_range(c, a, lo, hi, sample, samp, last, w.Dh, lo, f))) return rc;
    }
    return ev_end(c);
}

// The actions of the checkpointing schedule on the GPU: background
// restores, advances and history recomputation on the forward tiling, the
// adjoint with the fused imaging condition on the adjoint tiling.
struct SweepOps {
    fwi_ctx *c;
    Sweep &w;
    StepArgs af, a;
    float *inj;
    Fields f, fa;
    int seg_lo(int q) const { return q * w.k; }
    int seg_hi(int q) const { return std::min(c->plan.nt_max, (q + 1) * w.k); }
    int restore(int slot, int)
    {
        const Plan &p = c->plan;
        const int64_t ff = p.field_floats;
        hipStream_t st = c->stream;
        float *P = psi_block(c, PSI_FWD);
        if (slot < 0) {
            int rc = other(c, launch_fill(w.F[0], 2 * ff, 0.f, st), "fill");
            if (!rc && P) rc = other(c, launch_fill(P, 2 * ff, 0.f, st), "fill");
            if (rc) return rc;
        } else {
            const float *ckp = w.CK + size_t(slot) * snap_fields(p) * ff;
            HIPCHK(c, hipMemcpyAsync(w.F[0], ckp, size_t(ff) * 4, hipMemcpyDeviceToDevice, st));
            HIPCHK(c, hipMemcpyAsync(w.F[1], ckp + ff, size_t(ff) * 4, hipMemcpyDeviceToDevice, st));
            if (P) HIPCHK(c, hipMemcpyAsync(P, ckp + 2 * ff, size_t(2 * ff) * 4, hipMemcpyDeviceToDevice, st));
        }
        f = with_psi(Fields{w.F[0], w.F[1], w.F[2], w.F[3]}, P, ff);
        return FWI_OK;
    }
    int store(int slot, int)
    {
        const Plan &p = c->plan;
        const int64_t ff = p.field_floats;
        float *ckp = w.CK + size_t(slot) * snap_fields(p) * ff;
        HIPCHK(c, hipMemcpyAsync(ckp, f.prev, size_t(ff) * 4, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(ckp + ff, f.cur, size_t(ff) * 4, hipMemcpyDeviceToDevice, c->stream));
        if (p.pml) {
            HIPCHK(c, hipMemcpyAsync(ckp + 2 * ff, f.px, size_t(ff) * 4, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(ckp + 3 * ff, f.pz, size_t(ff) * 4, hipMemcpyDeviceToDevice, c->stream));
        }
        return FWI_OK;
    }
    // one segment per time loop, so that the captured loops repeat
    int forward(int q, bool emit)
    {
        int rc;
        const int lo = seg_lo(q), hi = seg_hi(q);
        if ((rc = ev_begin(c, K_FWD))) return rc;
        if ((rc = forward_range(c, af, lo, hi, false, nullptr, emit, w.Dh, lo, f))) return rc;
        c->stats.recomputed_steps += hi - lo;
        return ev_end(c);
    }
    int advance(int q0, int q1)
    {
        for (int q = q0; q < q1; ++q) {
            const int rc = forward(q, false);
            if (rc) return rc;
        }
        return FWI_OK;
    }
    int emit(int q) { return forward(q, true); }
    int adjoint(int q)
    {
        int rc;
        const Plan &p = c->plan;
        const int64_t gf = p.img_floats;
        const int lo = seg_lo(q), hi = seg_hi(q);
        const bool two = c->tile[K_ADJ].tb == 2;
        if ((rc = ev_begin(c, K_ADJ))) return rc;
        std::vector<char> key;
        key_put(key, 'A');
        key_put(key, a);
        key_put(key, lo);
        key_put(key, hi);
        key_put(key, w.Dh);
        key_put(key, inj);
        key_put(key, fa);
        rc = run_loop(c, key, fa, [&](Fields &ff) {
            StepArgs b = a;
            for (int n = hi - 1; n >= lo;) {
                const int levels = (two && n - 1 >= lo) ? 2 : 1;
                b.n = n;
                b.n2 = n - 1;
                b.dslot = w.Dh + size_t(n - lo) * gf;
                b.inj = inj + size_t(n) * p.Q;
                if (levels == 2) {
                    b.dslot2 = w.Dh + size_t(n - 1 - lo) * gf;
                    b.inj2 = inj + size_t(n - 1) * p.Q;
                }
                // a pair takes the shots alive at its second (earlier) level
                const int r = step_launch(c, b, K_ADJ, F_INJECT | F_IMAGE, levels, n - levels + 1, ff);
                if (r) return r;
                n -= levels;
            }
            return int(FWI_OK);
        });
        if (rc) return rc;
        return ev_end(c);
    }
};

// Backward sweep: the segments last to first, each one's D^n history
// recomputed from a snapshot by the checkpointing schedule (the last one's
// is already stored), the adjoint steps with the fused imaging condition
// run over it; finally fold and scale the image. The adjoint sources
// (time-major [nt_max][Q]) are in the samples buffer.
int backward_sweep(fwi_ctx *c, const float *v, Sweep &w, float *img)
{
    const Plan &p = c->plan;
    const int64_t ff = p.field_floats, gf = p.img_floats;
    hipStream_t st = c->stream;
    int rc;
    if ((rc = other(c, launch_fill(w.A[0], 4 * ff, 0.f, st), "fill"))) return rc;
    if ((rc = other(c, launch_fill(w.G, gf, 0.f, st), "fill"))) return rc;
    if ((rc = ensure_psi(c)) || (rc = zero_psi(c, PSI_ADJ))) return rc;
    SweepOps ops{c, w, base_args(c, v, K_FWD), base_args(c, v, K_ADJ), static_cast<float *>(c->samples.p),
                 with_psi(Fields{w.F[0], w.F[1], w.F[2], w.F[3]}, psi_block(c, PSI_FWD), ff),
                 // lambda^{n+2} (prev) and lambda^{n+1} (cur), both zero at the start
                 with_psi(Fields{w.A[0], w.A[1], w.A[2], w.A[3]}, psi_block(c, PSI_ADJ), ff)};
    ops.a.G = w.G;
    std::vector<int> free = revolve_free(w.slots);
    if ((rc = revolve(ops, w.nseg, 0, w.nseg, -1, free))) return rc;
    FinalArgs fin{};
    fin.shots = static_cast<const ShotDesc *>(c->d_shots.p);
    fin.nshots = p.S;
    fin.G = w.G;
    fin.v = v;
    fin.nz = p.nz;
    fin.nx = p.nx;
    fin.nb = p.nb;
    fin.top = p.top;
    fin.rel = p.relative ? 1 : 0;
    fin.NZ = p.NZ;
    fin.dt2 = float(double(p.dt) * p.dt);
    fin.img = img;
    int max_nx = 0;
    for (const ShotDesc &d : p.shots) max_nx = std::max(max_nx, d.NX);
    return other(c, launch_finalize(fin, max_nx, st), "finalize");
}

TraceArgs trace_args(fwi_ctx *c)
{
    const Plan &p = c->plan;
    TraceArgs t{};
    t.Q = p.Q;
    t.nt_max = p.nt_max;
    t.q_nt = static_cast<const int32_t *>(c->d_qnt.p);
    t.q_rptr = static_cast<const int32_t *>(c->d_qrptr.p);
    t.q_roff = static_cast<const int64_t *>(c->d_qroff.p);
    t.ndata = p.data_size;
    if (p.offgrid) {
        t.offgrid = 1;
        t.R = p.nrec;
        t.r_cptr = static_cast<const int32_t *>(c->d_rcptr.p);
        t.r_cq = static_cast<const int32_t *>(c->d_rcq.p);
        t.r_nt = static_cast<const int32_t *>(c->d_rnt.p);
        t.r_cw = static_cast<const float *>(c->d_rcw.p);
        t.q_rw = static_cast<const float *>(c->d_qrw.p);
        t.r_off = static_cast<const int64_t *>(c->d_roff.p);
        t.resid = static_cast<float *>(c->resid.p);
    }
    return t;
}

// ---- autotuner ----------------------------------------------------------------
//
// Picks, per kernel class, the strip width (64 or 128 columns: 1 or 2
// columns per lane) and the rows one wave streams, by timing a few launches
// of each candidate on the plan's real shapes. Runs once per plan (the
// plan cache keeps the result) on zeroed scratch fields; timings do not
// depend on the field values.

struct Candidate {
    int cw, rows, tb, pd;
};
// one level per launch: short row runs keep many waves in flight, a deeper
// prefetch more bytes per wave; two levels per launch recompute 4 rows above
// and below each run, so runs are longer (short runs still pay where a grid
// holds few waves)
const Candidate kTune[] = {
    {1, 8, 1, 1},  {1, 16, 1, 1}, {1, 24, 1, 1}, {1, 32, 1, 1}, {1, 48, 1, 1}, {2, 8, 1, 1},  {2, 16, 1, 1},
    {2, 24, 1, 1}, {2, 32, 1, 1}, {1, 8, 1, 2},  {1, 16, 1, 2}, {1, 24, 1, 2}, {1, 32, 1, 2}, {1, 48, 1, 2},
    {2, 8, 1, 2},  {2, 16, 1, 2}, {2, 24, 1, 2}, {2, 32, 1, 2}, {1, 24, 2, 1}, {1, 48, 2, 1}, {2, 24, 2, 1},
    {2, 48, 2, 1}, {1, 24, 2, 2}, {1, 48, 2, 2}, {1, 96, 2, 2}, {2, 24, 2, 2}, {2, 48, 2, 2}, {2, 96, 2, 2},
    {1, 16, 2, 1}, {1, 16, 2, 2}, {2, 16, 2, 2}, {1, 32, 2, 2}, {2, 32, 2, 2}};

constexpr int kTuneLaunches = 10;   // timed launches per candidate and pass
constexpr int kTunePasses = 2;      // passes over the list; the best time counts
// D slots the trial launches cycle through, as a real sweep streams through
// its history: together larger than the last-level cache, so D moves to and
// from HBM as it does in a real sweep
constexpr int kTuneSlots = 12;

// time of one time level of kernel class `cls` with tiling t (ms per level)
int time_class(fwi_ctx *c, int cls, const Tiling &t, const float *v, float *ms_out)
{
    const Plan &p = c->plan;
    const int64_t ff = p.field_floats, gf = p.img_floats;
    float *F = static_cast<float *>(c->fields.p);
    StepArgs b = base_args(c, v, cls);
    b.waves = static_cast<const WaveDesc *>(t.d_waves.p);
    b.rrows = static_cast<const RecRow *>(t.d_rrows.p);
    b.rmap = static_cast<const int32_t *>(t.d_rmap.p);
    b.cw = t.cw;
    b.pd = t.pd;
    b.n = 1;
    b.n2 = cls == K_ADJ ? 0 : 2;
    b.nwaves = t.prefix[p.active_slots(std::min(b.n, b.n2))];
    b.cur = F;
    b.prev = F + ff;
    b.out1 = F + 2 * ff;
    b.out2 = F + 3 * ff;
    b.cur2 = F + 2 * ff;
    b.prev2 = F + 3 * ff;
    b.dv = v;
    float *const dhist = static_cast<float *>(c->dhist.p);
    b.dslot = dhist;
    b.dslot2 = dhist + gf;
    b.G = static_cast<float *>(c->image.p);
    b.samp = static_cast<float *>(c->samples.p);
    b.samp2 = b.samp + p.Q;
    b.inj = b.samp;
    b.inj2 = b.samp2;
    if (float *P = psi_block(c, PSI_FWD)) {   // zeroed trial edge fields
        float *Q = psi_block(c, PSI_SCAT);
        b.psx_in = P;
        b.psz_in = P + ff;
        b.psx_out = P + 2 * ff;
        b.psz_out = P + 3 * ff;
        b.psx2_in = Q;
        b.psz2_in = Q + ff;
        b.psx2_out = Q + 2 * ff;
        b.psz2_out = Q + 3 * ff;
    }
    // the forward class is timed as the forward of a gradient or migration
    // (emitting D), its most frequent and heaviest form
    const int flags = cls == K_ADJ ? (F_INJECT | F_IMAGE) : (F_SRC | F_SAMPLE | F_EMIT);
    int slot = 0;
    auto launch = [&]() -> hipError_t {
        b.dslot = dhist + int64_t(slot) * gf;
        b.dslot2 = b.dslot + gf;
        slot = (slot + 1) % kTuneSlots;
        if (cls == K_BORN) {
            b.dslot = nullptr;   // the Born step of a demigration (no D output)
            return launch_born_step(b, c->stream);
        }
        const int fl = cls == K_SCAT ? (F_SAMPLE | F_SCAT) : flags;
        return t.tb == 2 ? launch_step2(fl, b, c->stream) : launch_step(fl, b, c->stream);
    };
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    hipError_t err = launch();
    if (err == hipSuccess) err = launch();
    if (err == hipSuccess) err = hipEventRecord(e0, c->stream);
    for (int i = 0; i < kTuneLaunches && err == hipSuccess; ++i) err = launch();
    if (err == hipSuccess) err = hipEventRecord(e1, c->stream);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return set_err(c, FWI_EHIP, "autotune launch: %s", hipGetErrorString(err));
    *ms_out = ms / float(kTuneLaunches * t.tb);
    return FWI_OK;
}

int ensure_tilings(fwi_ctx *c, const float *v)
{
    const Plan &p = c->plan;
    bool need_tune = false;
    for (int k = 0; k < kClasses; ++k) {
        Tiling &t = c->tile[k];
        const bool forced = c->force_cw[k] != 0;
        const int want_cw = forced ? c->force_cw[k] : (c->autotune ? 0 : kDefaultCw);
        const int want_rows = forced ? c->force_rows[k] : (c->autotune ? 0 : kDefaultRows);
        const int want_tb = one_level(k) ? 1 : (forced ? c->force_tb[k] : (c->autotune ? 0 : kDefaultTb));
        const int want_pd = forced ? c->force_pd[k] : kDefaultPd;
        if (want_cw && want_rows && want_tb) {
            if (t.cw == want_cw && t.rows == want_rows && t.tb == want_tb && t.pd == want_pd) continue;
            clear_graphs(c);
            build_tiling(p, want_cw, want_rows, want_tb, want_pd, t);
            int rc = upload_tiling(c, t);
            if (rc) return rc;
        } else if (t.cw == 0) {
            need_tune = true;
        }
    }
    if (!need_tune) return FWI_OK;
    clear_graphs(c);
    // scratch for the trial launches (two levels: four fields, two D slots,
    // two sample rows)
    const int64_t ff = p.field_floats, gf = p.img_floats;
    const int64_t nq = 2 * std::max(p.Q, 1);
    int rc = FWI_OK;
    if ((rc = ensure(c, c->fields, size_t(4 * ff) * 4)) || (rc = ensure(c, c->image, size_t(gf) * 4)) ||
        (rc = ensure(c, c->dhist, size_t((kTuneSlots + 1) * gf) * 4)) ||
        (rc = ensure(c, c->samples, size_t(nq) * 4)) || (rc = ensure_psi(c)) || (rc = zero_psi(c, PSI_FWD)) ||
        (rc = zero_psi(c, PSI_SCAT)))
        return rc;
    if ((rc = other(c, launch_fill(static_cast<float *>(c->fields.p), 4 * ff, 0.f, c->stream), "fill")) ||
        (rc = other(c, launch_fill(static_cast<float *>(c->image.p), gf, 0.f, c->stream), "fill")) ||
        (rc = other(c, launch_fill(static_cast<float *>(c->dhist.p), (kTuneSlots + 1) * gf, 0.f, c->stream),
                    "fill")) ||
        (rc = other(c, launch_fill(static_cast<float *>(c->samples.p), nq, 0.f, c->stream), "fill")))
        return rc;
    float best[kClasses];
    Candidate bc[kClasses];
    for (int k = 0; k < kClasses; ++k) {
        best[k] = 1e30f;
        bc[k] = {kDefaultCw, kDefaultRows, one_level(k) ? 1 : kDefaultTb, kDefaultPd};
    }
    Tiling trial;
    for (int pass = 0; pass < kTunePasses && rc == 0; ++pass) {
        for (const Candidate &cand : kTune) {
            build_tiling(p, cand.cw, cand.rows, cand.tb, cand.pd, trial);
            if ((rc = upload_tiling(c, trial))) break;
            for (int k = 0; k < kClasses; ++k) {
                if (c->tile[k].cw != 0 || (one_level(k) && cand.tb != 1) ||
                    (k == K_BORN && cand.pd != 1))
                    continue;
                float ms = 0.f;
                if ((rc = time_class(c, k, trial, v, &ms))) break;
                if (ms < best[k]) {
                    best[k] = ms;
                    bc[k] = cand;
                }
            }
            if (rc) break;
        }
    }
    trial.release_all();
    if (rc) return rc;
    for (int k = 0; k < kClasses; ++k) {
        Tiling &t = c->tile[k];
        if (t.cw != 0) continue;
        build_tiling(p, bc[k].cw, bc[k].rows, bc[k].tb, bc[k].pd, t);
        if ((rc = upload_tiling(c, t))) return rc;
    }
    return FWI_OK;
}

int begin_call(fwi_ctx *c, const fwi_grid *g, const fwi_geom *geo)
{
    if (!c) return FWI_EINVAL;
    c->err.clear();
    reset_stats(c);
    c->ev_marks.clear();
    c->ev_used = 0;
    HIPCHK(c, hipSetDevice(c->device));
    return build_plan(c, g, geo);
}

// Tilings are (re)built after the model check, which the trial launches
// need (they read the model).
int prepare(fwi_ctx *c, const float *v)
{
    int rc = ensure_tilings(c, v);
    if (rc) return rc;
    for (int k = 0; k < kClasses; ++k) {
        c->stats.tile_cw[k] = c->tile[k].cw;
        c->stats.tile_rows[k] = c->tile[k].rows;
        c->stats.tile_levels[k] = c->tile[k].tb;
        c->stats.tile_prefetch[k] = c->tile[k].pd;
    }
    return FWI_OK;
}

int forward_sweep_sampled(fwi_ctx *c, const float *v)
{
    const Plan &p = c->plan;
    const int64_t ff = p.field_floats;
    int rc;
    if ((rc = ensure(c, c->fields, size_t(4 * ff) * 4)) ||
        (rc = ensure(c, c->samples, size_t(p.nt_max) * p.Q * 4)) || (rc = ensure_psi(c)))
        return rc;
    float *F = static_cast<float *>(c->fields.p);
    float *samp = static_cast<float *>(c->samples.p);
    if ((rc = other(c, launch_fill(F, 4 * ff, 0.f, c->stream), "fill")) || (rc = zero_psi(c, PSI_FWD))) return rc;
    StepArgs a = base_args(c, v, K_FWD);
    Fields f = with_psi(Fields{F, F + ff, F + 2 * ff, F + 3 * ff}, psi_block(c, PSI_FWD), ff);
    if ((rc = ev_begin(c, K_FWD))) return rc;
    if ((rc = forward_range(c, a, 0, p.nt_max, true, samp, false, nullptr, 0, f))) return rc;
    return ev_end(c);
}

// Joint Born steps lo .. hi-1 (background u in U0/U1, scattered du in
// D0/D1, alternating by step parity); du samples to samp + n*Q; with dh the
// background's D^n goes to slot n - dlo of dh.
int born_range(fwi_ctx *c, const StepArgs &a, int lo, int hi, float *samp, float *dh, int dlo, float *U0, float *U1,
               float *D0, float *D1)
{
    if (lo >= hi) return FWI_OK;
    const Plan &p = c->plan;
    const int64_t gf = p.img_floats;
    std::vector<char> key;
    key_put(key, 'B');
    key_put(key, a);
    key_put(key, lo);
    key_put(key, hi);
    key_put(key, samp);
    key_put(key, dh);
    key_put(key, dlo);
    key_put(key, U0);
    key_put(key, U1);
    key_put(key, D0);
    key_put(key, D1);
    key_put(key, c->psi.p);
    Fields none{};
    // the layer's edge fields alternate by step parity as the fields do
    float *PU = psi_block(c, PSI_FWD), *PD = psi_block(c, PSI_SCAT);
    const int64_t ff = p.field_floats;
    return run_loop(c, key, none, [&](Fields &) {
        StepArgs b = a;
        for (int n = lo; n < hi; ++n) {
            b.n = n;
            b.nwaves = c->tile[K_BORN].prefix[p.active_slots(n)];
            b.cur = n % 2 == 0 ? U0 : U1;
            b.prev = n % 2 == 0 ? U1 : U0;
            b.cur2 = n % 2 == 0 ? D0 : D1;
            b.prev2 = n % 2 == 0 ? D1 : D0;
            if (PU) {
                const int64_t i = n % 2 == 0 ? 0 : 2 * ff, o = n % 2 == 0 ? 2 * ff : 0;
                b.psx_in = PU + i;
                b.psz_in = PU + i + ff;
                b.psx_out = PU + o;
                b.psz_out = PU + o + ff;
                b.psx2_in = PD + i;
                b.psz2_in = PD + i + ff;
                b.psx2_out = PD + o;
                b.psz2_out = PD + o + ff;
            }
            b.samp = samp + size_t(n) * p.Q;
            b.dslot = dh ? dh + size_t(n - dlo) * gf : nullptr;
            HIPCHK(c, launch_born_step(b, c->stream));
            const double upd = step_updates(p, n);
            c->stats.cell_updates += 2 * upd;
            c->stats.stencil_launches += 1;
            c->stats.n_born += 1;
            c->stats.bytes_born += upd * (kBytesBorn + (dh ? kBytesEmit : 0.0));
        }
        return int(FWI_OK);
    });
}

// The FWI gradient after begin_call: leaves the sweep state (and, with one
// segment, the whole D^n history) in the context.
int gradient_core(fwi_ctx *c, const float *v, const float *d_obs, float *grad, double *misfit, float *d_syn,
                  Sweep &w)
{
    int rc;
    const Plan &p = c->plan;
    if (!grad) return set_err(c, FWI_EINVAL, "g is NULL");
    if (!d_obs && p.data_size > 0) return set_err(c, FWI_EINVAL, "d_obs is NULL");
    if ((rc = check_model(c, v, "v")) || (rc = prepare(c, v))) return rc;
    // forward with sampling and checkpoints, then the residual (in place
    // over the samples), then the backward sweep
    if ((rc = forward_for_adjoint(c, v, true, w))) return rc;
    TraceArgs t = trace_args(c);
    float *samp = static_cast<float *>(c->samples.p);
    t.tm_in = samp;
    t.alpha = 1.f;
    t.tr_in = d_obs;
    t.beta = -1.f;
    t.tm_out = samp;
    t.tr_out = d_syn;
    const int64_t nmax = traces_partials_max(p.Q, p.nt_max);
    if ((rc = ensure(c, c->partials, size_t(std::max<int64_t>(nmax, 1)) * sizeof(double))) ||
        (rc = ensure(c, c->misfit, sizeof(double))))
        return rc;
    t.partials = static_cast<double *>(c->partials.p);
    int64_t nblk = 0;
    if ((rc = other(c, launch_traces(t, c->stream, &nblk), "residual"))) return rc;
    if (nblk > 0) {
        if ((rc = other(c, launch_sum_partials(t.partials, nblk, static_cast<double *>(c->misfit.p), c->stream),
                        "misfit")))
            return rc;
    } else {
        HIPCHK(c, hipMemsetAsync(c->misfit.p, 0, sizeof(double), c->stream));
    }
    if (misfit)
        HIPCHK(c, hipMemcpyAsync(c->h_misfit, c->misfit.p, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if ((rc = backward_sweep(c, v, w, grad))) return rc;
    if (misfit) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        *misfit = *c->h_misfit;
    }
    return FWI_OK;
}

// The pair after the model and perturbation are in the context (v0, dv are
// the context copies) and the tilings are prepared.
int pair_core(fwi_ctx *c, const float *v0, const float *dv, float *dd, float *img)
{
    int rc;
    const Plan &p = c->plan;
    Sweep w;
    if ((rc = choose_segments(c, w))) return rc;
    const int k = w.k, nseg = w.nseg;
    const int64_t ff = p.field_floats, gf = p.img_floats;
    const int sf = snap_fields(p);
    if ((rc = ensure(c, c->fields, size_t(8 * ff) * 4)) || (rc = ensure(c, c->image, size_t(gf) * 4)) ||
        (rc = ensure(c, c->dhist, size_t(k) * gf * 4)) ||
        (rc = ensure(c, c->ckpt, size_t(w.slots) * sf * ff * 4)) ||
        (rc = ensure(c, c->samples, size_t(p.nt_max) * p.Q * 4)) || (rc = ensure_psi(c)) ||
        (!dd && (rc = ensure(c, c->pairdata, size_t(std::max<int64_t>(p.data_size, 1)) * 4))))
        return rc;
    float *F = static_cast<float *>(c->fields.p);
    for (int i = 0; i < 4; ++i) {
        w.F[i] = F + i * ff;
        w.A[i] = F + (4 + i) * ff;
    }
    w.Dh = static_cast<float *>(c->dhist.p);
    w.CK = static_cast<float *>(c->ckpt.p);
    w.G = static_cast<float *>(c->image.p);
    float *samp = static_cast<float *>(c->samples.p);
    hipStream_t st = c->stream;
    if ((rc = other(c, launch_fill(w.F[0], 4 * ff, 0.f, st), "fill")) || (rc = zero_psi(c, PSI_FWD)) ||
        (rc = zero_psi(c, PSI_SCAT)))
        return rc;
    StepArgs a = base_args(c, v0, K_BORN);
    a.dv = dv;
    float *U0 = w.F[0], *U1 = w.F[1], *D0 = w.F[2], *D1 = w.F[3];
    float *PU = psi_block(c, PSI_FWD);
    if ((rc = ev_begin(c, K_BORN))) return rc;
    for (int sgi = 0; sgi < nseg; ++sgi) {
        const int lo = sgi * k, hi = std::min(p.nt_max, lo + k);
        const bool last = sgi == nseg - 1;
        if (w.spine[size_t(sgi)] >= 0) {
            // (u^{lo-1}, u^lo): the fields the step at n = lo reads as prev,
            // cur (and the edge fields it reads)
            float *ckp = w.CK + size_t(w.spine[size_t(sgi)]) * sf * ff;
            HIPCHK(c, hipMemcpyAsync(ckp, lo % 2 == 0 ? U1 : U0, size_t(ff) * 4, hipMemcpyDeviceToDevice, st));
            HIPCHK(c, hipMemcpyAsync(ckp + ff, lo % 2 == 0 ? U0 : U1, size_t(ff) * 4, hipMemcpyDeviceToDevice, st));
            if (PU)
                HIPCHK(c, hipMemcpyAsync(ckp + 2 * ff, PU + (lo % 2 == 0 ? 0 : 2 * ff), size_t(2 * ff) * 4,
                                         hipMemcpyDeviceToDevice, st));
        }
        if ((rc = born_range(c, a, lo, hi, samp, last ? w.Dh : nullptr, lo, U0, U1, D0, D1))) return rc;
    }
    if ((rc = ev_end(c))) return rc;
    // samples -> packed data J dv -> adjoint sources (co-located receivers add)
    float *data = dd ? dd : static_cast<float *>(c->pairdata.p);
    TraceArgs t = trace_args(c);
    t.tm_in = samp;
    t.alpha = 1.f;
    t.tr_out = data;
    if ((rc = other(c, launch_traces(t, st, nullptr), "traces"))) return rc;
    TraceArgs t2 = trace_args(c);
    t2.tr_in = data;
    t2.beta = 1.f;
    t2.tm_out = samp;
    if ((rc = other(c, launch_traces(t2, st, nullptr), "adjoint sources"))) return rc;
    return backward_sweep(c, v0, w, img);
}

// Scattered-field steps lo .. hi-1 with the source (2 dV / V) D^n read from
// slot n - dlo of dh (the stored background history); du^{n+1} samples to
// samp + n*Q. Pairs of levels per launch when the class's tiling runs two.
int scat_range(fwi_ctx *c, const StepArgs &a, int lo, int hi, float *samp, float *dh, int dlo, Fields &f)
{
    if (lo >= hi) return FWI_OK;
    const Plan &p = c->plan;
    const int64_t gf = p.img_floats;
    std::vector<char> key;
    key_put(key, 'S');
    key_put(key, a);
    key_put(key, lo);
    key_put(key, hi);
    key_put(key, samp);
    key_put(key, dh);
    key_put(key, dlo);
    key_put(key, f);
    const bool two = c->tile[K_SCAT].tb == 2;
    return run_loop(c, key, f, [&](Fields &ff) {
        StepArgs b = a;
        int rc;
        for (int n = lo; n < hi;) {
            const int levels = (two && n + 1 < hi) ? 2 : 1;
            b.n = n;
            b.n2 = n + 1;
            b.samp = samp + size_t(n) * p.Q;
            b.samp2 = samp + size_t(n + 1) * p.Q;
            b.dslot = dh + size_t(n - dlo) * gf;
            b.dslot2 = dh + size_t(n + 1 - dlo) * gf;
            if ((rc = step_launch(c, b, K_SCAT, F_SAMPLE | F_SCAT, levels, n, ff))) return rc;
            n += levels;
        }
        return int(FWI_OK);
    });
}

// An allocation-free call runs on a set-aside copy of the context: every
// device buffer, the plan, the tilings and the captured loops of the
// context are moved out for the call and moved back afterwards (the call's
// own buffers, carved from the static scratch, are then dropped), so the
// context is left as it was. Inside, ensure() carves instead of allocating,
// and graph capture, profiling events and the autotuner (which create HIP
// objects) are off: the tiling is the forced one or the fixed default, and
// every tiling gives the same bits.
class ArenaScope {
   public:
    explicit ArenaScope(fwi_ctx *c) : c_(c)
    {
        for (size_t i = 0; i < kBufs; ++i) {
            saved_[i] = *bufs()[i];
            *bufs()[i] = DevBuf{};
        }
        plan_ = std::move(c->plan);
        c->plan = Plan{};
        plan_valid_ = c->plan_valid;
        c->plan_valid = false;
        for (int k = 0; k < kClasses; ++k) {
            tile_[k] = std::move(c->tile[k]);
            c->tile[k] = Tiling{};
        }
        graphs_cache_ = std::move(c->graph_cache);
        c->graph_cache.clear();
        graphs_ = c->graphs;
        profiling_ = c->profiling;
        autotune_ = c->autotune;
        c->graphs = c->profiling = c->autotune = false;
        c->arena = c->scratch_dev;
        c->arena_used = 0;
    }
    ~ArenaScope()
    {
        fwi_ctx *c = c_;
        c->arena = nullptr;
        c->arena_used = 0;
        for (size_t i = 0; i < kBufs; ++i) *bufs()[i] = saved_[i];
        c->plan = std::move(plan_);
        c->plan_valid = plan_valid_;
        for (int k = 0; k < kClasses; ++k) c->tile[k] = std::move(tile_[k]);
        c->graph_cache = std::move(graphs_cache_);
        c->graphs = graphs_;
        c->profiling = profiling_;
        c->autotune = autotune_;
    }
    ArenaScope(const ArenaScope &) = delete;
    ArenaScope &operator=(const ArenaScope &) = delete;

   private:
    static constexpr size_t kBufs = 24;
    std::array<DevBuf *, kBufs> bufs()
    {
        fwi_ctx *c = c_;
        return {&c->d_shots, &c->d_qnt, &c->d_qrptr, &c->d_qroff, &c->d_wav, &c->d_qrw, &c->d_rcptr, &c->d_rcq,
                &c->d_rnt, &c->d_rcw, &c->d_roff, &c->fields, &c->samples, &c->image, &c->dhist, &c->ckpt,
                &c->partials, &c->misfit, &c->check, &c->pairdata, &c->resid, &c->model, &c->dmodel, &c->psi};
    }
    fwi_ctx *c_;
    DevBuf saved_[kBufs];
    Plan plan_;
    bool plan_valid_ = false;
    Tiling tile_[kClasses];
    std::vector<GraphEntry> graphs_cache_;
    bool graphs_ = true, profiling_ = false, autotune_ = true;
};

}  // namespace

namespace fwi {
hipStream_t ctx_stream(const fwi_ctx *c) { return c->stream; }
int ctx_device(const fwi_ctx *c) { return c->device; }
}  // namespace fwi

// ===========================================================================
// public entry points

extern "C" {

int fwi_ctx_create(int device, void *hip_stream, fwi_ctx **out)
{
    if (!out) return FWI_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FWI_EHIP;
    if (hipSetDevice(device) != hipSuccess) return FWI_EHIP;
    fwi_ctx *c = new fwi_ctx();
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) tot = size_t(64) << 30;
    c->budget = int64_t(kDefaultBudgetFrac * double(tot));
    if (hipHostMalloc(reinterpret_cast<void **>(&c->h_check), 4 * sizeof(float), hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&c->h_misfit), sizeof(double), hipHostMallocDefault) !=
            hipSuccess) {
        fwi_ctx_destroy(c);
        return FWI_ENOMEM;
    }
    if (scratch_address(device, &c->scratch_dev) != FWI_OK) {
        fwi_ctx_destroy(c);
        return FWI_EHIP;
    }
    *out = c;
    return FWI_OK;
}

void fwi_ctx_destroy(fwi_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (Tiling &t : c->tile) t.release_all();
    for (DevBuf *b : {&c->d_qrw, &c->d_rcptr, &c->d_rcq, &c->d_rnt, &c->d_rcw, &c->d_roff, &c->resid, &c->psi})
        release(*b);
    for (DevBuf *b : {&c->d_shots, &c->d_qnt, &c->d_qrptr, &c->d_qroff, &c->d_wav, &c->fields, &c->samples,
                      &c->image, &c->dhist, &c->ckpt, &c->partials, &c->misfit, &c->check, &c->model, &c->dmodel,
                      &c->pairdata, &c->rtm_data, &c->rtm_img, &c->d_mute_off, &c->d_mute_nt, &c->d_mute_t0})
        release(*b);
    clear_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    if (c->h_check) (void)hipHostFree(c->h_check);
    if (c->h_misfit) (void)hipHostFree(c->h_misfit);
    delete c;
}

int fwi_ctx_set_stream(fwi_ctx *c, void *hip_stream)
{
    if (!c) return FWI_EINVAL;
    c->stream = static_cast<hipStream_t>(hip_stream);
    return FWI_OK;
}

int fwi_ctx_set_ckpt_slots(fwi_ctx *c, int32_t slots)
{
    if (!c) return FWI_EINVAL;
    if (slots < -1) return set_err(c, FWI_EINVAL, "ckpt slots must be >= -1");
    c->ckpt_slots = slots;
    return FWI_OK;
}

int fwi_checkpoint_schedule(int32_t nseg, int32_t slots, int64_t *recomputed)
{
    return revolve_check(nseg, slots, recomputed);
}

int fwi_ctx_set_mem_budget(fwi_ctx *c, int64_t bytes)
{
    if (!c || bytes < 0) return FWI_EINVAL;
    if (bytes == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) tot = size_t(64) << 30;
        bytes = int64_t(kDefaultBudgetFrac * double(tot));
    }
    c->budget = bytes;
    return FWI_OK;
}

int fwi_ctx_set_profiling(fwi_ctx *c, int enable)
{
    if (!c) return FWI_EINVAL;
    c->profiling = enable != 0;
    return FWI_OK;
}

int fwi_ctx_set_tiling(fwi_ctx *c, int kernel, int cols_per_lane, int rows_per_wave, int levels_per_launch,
                       int prefetch_rows)
{
    if (!c || kernel < -1 || kernel >= kClasses) return FWI_EINVAL;
    const bool reset = cols_per_lane == 0 && rows_per_wave == 0 && levels_per_launch == 0;
    if (!reset && !((cols_per_lane == 1 || cols_per_lane == 2) && rows_per_wave >= 1 && rows_per_wave <= 4096 &&
                    (levels_per_launch == 1 || levels_per_launch == 2) && prefetch_rows >= 0 &&
                    prefetch_rows <= 2))
        return FWI_EINVAL;
    // the joint Born kernel runs one level per launch
    if (kernel >= 0 && one_level(kernel) && levels_per_launch == 2) return FWI_EINVAL;
    for (int k = 0; k < kClasses; ++k)
        if (kernel == -1 || kernel == k) {
            c->force_cw[k] = cols_per_lane;
            c->force_rows[k] = rows_per_wave;
            c->force_tb[k] = one_level(k) && !reset ? 1 : levels_per_launch;
            // the Born kernel prefetches one row ahead; the two-level kernel
            // one unless told otherwise
            c->force_pd[k] = k == K_BORN ? 1
                             : prefetch_rows ? prefetch_rows
                             : levels_per_launch == 2 ? 1 : kDefaultPd;
            c->tile[k].cw = c->tile[k].rows = c->tile[k].tb = 0;
        }
    return FWI_OK;
}

int fwi_ctx_set_autotune(fwi_ctx *c, int enable)
{
    if (!c) return FWI_EINVAL;
    c->autotune = enable != 0;
    for (int k = 0; k < kClasses; ++k)
        if (!c->force_cw[k]) c->tile[k].cw = c->tile[k].rows = c->tile[k].tb = 0;
    return FWI_OK;
}

int fwi_ctx_get_stats(const fwi_ctx *c, fwi_stats *out)
{
    if (!c || !out) return FWI_EINVAL;
    *out = c->stats;
    return FWI_OK;
}

int fwi_ctx_trim(fwi_ctx *c)
{
    if (!c) return FWI_EINVAL;
    (void)hipSetDevice(c->device);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return FWI_EHIP;
    clear_graphs(c);
    for (DevBuf *b : {&c->fields, &c->samples, &c->image, &c->dhist, &c->ckpt, &c->partials, &c->model, &c->dmodel,
                      &c->pairdata, &c->psi, &c->rtm_data, &c->rtm_img})
        release(*b);
    return FWI_OK;
}

int fwi_ctx_set_graphs(fwi_ctx *c, int enable)
{
    if (!c) return FWI_EINVAL;
    (void)hipSetDevice(c->device);
    if (!enable) {
        if (hipStreamSynchronize(c->stream) != hipSuccess) return FWI_EHIP;
        clear_graphs(c);
    }
    c->graphs = enable != 0;
    return FWI_OK;
}

const char *fwi_last_error(const fwi_ctx *c)
{
    return c ? c->err.c_str() : "NULL context";
}

int fwi_forward(fwi_ctx *c, const fwi_grid *g, const fwi_geom *geo, const float *v, float *d)
{
    int rc = begin_call(c, g, geo);
    if (rc) return rc;
    const Plan &p = c->plan;
    if (!d && p.data_size > 0) return set_err(c, FWI_EINVAL, "d is NULL");
    if ((rc = check_model(c, v, "v")) || (rc = prepare(c, v))) return rc;
    if ((rc = forward_sweep_sampled(c, v))) return rc;
    TraceArgs t = trace_args(c);
    t.tm_in = static_cast<const float *>(c->samples.p);
    t.alpha = 1.f;
    t.tr_out = d;
    if ((rc = other(c, launch_traces(t, c->stream, nullptr), "traces"))) return rc;
    return finish_stats(c);
}

int fwi_forward_noalloc(fwi_ctx *c, const fwi_grid *g, const fwi_geom *geo, const float *v, float *d)
{
    if (!c) return FWI_EINVAL;
    if (!c->scratch_dev) return set_err(c, FWI_ESTATE, "no scratch address on device %d", c->device);
    if (c->arena) return set_err(c, FWI_ESTATE, "allocation-free call inside another");
    ArenaScope scope(c);
    return fwi_forward(c, g, geo, v, d);
}

int fwi_gradient(fwi_ctx *c, const fwi_grid *g, const fwi_geom *geo, const float *v, const float *d_obs,
                 float *grad, double *misfit, float *d_syn)
{
    int rc = begin_call(c, g, geo);
    if (rc) return rc;
    Sweep w;
    if ((rc = gradient_core(c, v, d_obs, grad, misfit, d_syn, w))) return rc;
    return finish_stats(c);
}

int fwi_gradient_pair(fwi_ctx *c, const fwi_grid *g, const fwi_geom *geo, const float *v, const float *d_obs,
                      float *grad, double *misfit, float scale, float *img, float *dd)
{
    int rc = begin_call(c, g, geo);
    if (rc) return rc;
    if (!img) return set_err(c, FWI_EINVAL, "img is NULL");
    if (!(scale == scale) || std::isinf(scale)) return set_err(c, FWI_EINVAL, "scale must be finite");
    Sweep w;
    if ((rc = gradient_core(c, v, d_obs, grad, misfit, nullptr, w))) return rc;
    const Plan &p = c->plan;
    const float *mv = static_cast<const float *>(c->model.p);   // the call's model copy
    // dv = scale * g, in the context
    if ((rc = ensure(c, c->dmodel, size_t(p.nz) * p.nx * 4))) return rc;
    float *dv = static_cast<float *>(c->dmodel.p);
    if ((rc = other(c, launch_scale(grad, scale, dv, int64_t(p.nz) * p.nx, c->stream), "scale"))) return rc;
    if (w.nseg > 1) {
        // the history was checkpointed: the pair runs its own joint Born sweep
        if ((rc = pair_core(c, mv, dv, dd, img))) return rc;
        return finish_stats(c);
    }
    // the whole D^n history of the gradient's forward sweep is still stored:
    // only the scattered field is propagated, with the source (2 dV / V) D^n
    const int64_t ff = p.field_floats;
    float *samp = static_cast<float *>(c->samples.p);
    if (!dd && (rc = ensure(c, c->pairdata, size_t(std::max<int64_t>(p.data_size, 1)) * 4))) return rc;
    if ((rc = other(c, launch_fill(w.F[0], 2 * ff, 0.f, c->stream), "fill")) || (rc = zero_psi(c, PSI_SCAT)))
        return rc;
    StepArgs a = base_args(c, mv, K_SCAT);
    a.dv = dv;
    Fields f = with_psi(Fields{w.F[0], w.F[1], w.F[2], w.F[3]}, psi_block(c, PSI_SCAT), ff);
    if ((rc = ev_begin(c, K_BORN))) return rc;
    if ((rc = scat_range(c, a, 0, p.nt_max, samp, w.Dh, 0, f))) return rc;
    if ((rc = ev_end(c))) return rc;
    float *data = dd ? dd : static_cast<float *>(c->pairdata.p);
    TraceArgs t = trace_args(c);
    t.tm_in = samp;
    t.alpha = 1.f;
    t.tr_out = data;
    if ((rc = other(c, launch_traces(t, c->stream, nullptr), "traces"))) return rc;
    TraceArgs t2 = trace_args(c);
    t2.tr_in = data;
    t2.beta = 1.f;
    t2.tm_out = samp;
    if ((rc = other(c, launch_traces(t2, c->stream, nullptr), "adjoint sources"))) return rc;
    if ((rc = backward_sweep(c, mv, w, img))) return rc;
    return finish_stats(c);
}

int fwi_misfit(fwi_ctx *c, const fwi_grid *g, const fwi_geom *geo, const float *v, const float *d_obs,
               double *misfit)
{
    int rc = begin_call(c, g, geo);
    if (rc) return rc;
    const Plan &p = c->plan;
    if (!misfit) return set_err(c, FWI_EINVAL, "misfit is NULL");
    if (!d_obs && p.data_size > 0) return set_err(c, FWI_EINVAL, "d_obs is NULL");
    if ((rc = check_model(c, v, "v")) || (rc = prepare(c, v))) return rc;
    if ((rc = forward_sweep_sampled(c, v))) return rc;
    TraceArgs t = trace_args(c);
    t.tm_in = static_cast<const float *>(c->samples.p);
    t.alpha = 1.f;
    t.tr_in = d_obs;
    t.beta = -1.f;
    const int64_t nmax = traces_partials_max(p.Q, p.nt_max);
    if ((rc = ensure(c, c->partials, size_t(std::max<int64_t>(nmax, 1)) * sizeof(double))) ||
        (rc = ensure(c, c->misfit, sizeof(double))))
        return rc;
    t.partials = static_cast<double *>(c->partials.p);
    int64_t nblk = 0;
    if ((rc = other(c, launch_traces(t, c->stream, &nblk), "residual"))) return rc;
    if (nblk > 0) {
        if ((rc = other(c, launch_sum_partials(t.partials, nblk, static_cast<double *>(c->misfit.p), c->stream),
                        "misfit")))
            return rc;
    } else {
        HIPCHK(c, hipMemsetAsync(c->misfit.p, 0, sizeof(double), c->stream));
    }
    HIPCHK(c, hipMemcpyAsync(c->h_misfit, c->misfit.p, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *misfit = *c->h_misfit;
    return finish_stats(c);
}

int born_demig(fwi_ctx *c, const fwi_grid *g, const fwi_geom *geo, const float *v0, const float *dv, float *dd)
{
    int rc = begin_call(c, g, geo);
    if (rc) return rc;
    const Plan &p = c->plan;
    if (!dd && p.data_size > 0) return set_err(c, FWI_EINVAL, "dd is NULL");
    if ((rc = check_model(c, v0, "v0")) || (rc = check_perturbation(c, dv)) || (rc = prepare(c, v0)))
        return rc;
    const int64_t ff = p.field_floats;
    if ((rc = ensure(c, c->fields, size_t(4 * ff) * 4)) ||
        (rc = ensure(c, c->samples, size_t(p.nt_max) * p.Q * 4)) || (rc = ensure_psi(c)))
        return rc;
    float *F = static_cast<float *>(c->fields.p);
    float *samp = static_cast<float *>(c->samples.p);
    if ((rc = other(c, launch_fill(F, 4 * ff, 0.f, c->stream), "fill")) || (rc = zero_psi(c, PSI_FWD)) ||
        (rc = zero_psi(c, PSI_SCAT)))
        return rc;
    StepArgs a = base_args(c, v0, K_BORN);
    a.dv = dv;
    float *U0 = F, *U1 = F + ff, *D0 = F + 2 * ff, *D1 = F + 3 * ff;
    if ((rc = ev_begin(c, K_BORN))) return rc;
    if ((rc = born_range(c, a, 0, p.nt_max, samp, nullptr, 0, U0, U1, D0, D1))) return rc;
    if ((rc = ev_end(c))) return rc;
    TraceArgs t = trace_args(c);
    t.tm_in = samp;
    t.alpha = 1.f;
    t.tr_out = dd;
    if ((rc = other(c, launch_traces(t, c->stream, nullptr), "traces"))) return rc;
    return finish_stats(c);
}

// img = J^T J dv in one joint Born sweep: its background wavefield provides
// the imaging history (D^n of the last segment directly, checkpoints of
// (u^{n-1}, u^n) for the others), its scattered samples are the data J dv
// whose adjoint is then run. Equal to born_mig(born_demig(dv)) bit for bit
// without the migration's own background sweep.
int born_pair(fwi_ctx *c, const fwi_grid *g, const fwi_geom *geo, const float *v0, const float *dv, float *dd,
              float *img)
{
    int rc = begin_call(c, g, geo);
    if (rc) return rc;
    if (!img) return set_err(c, FWI_EINVAL, "img is NULL");
    if ((rc = check_model(c, v0, "v0")) || (rc = check_perturbation(c, dv)) || (rc = prepare(c, v0))) return rc;
    if ((rc = pair_core(c, v0, dv, dd, img))) return rc;
    return finish_stats(c);
}

int born_mig(fwi_ctx *c, const fwi_grid *g, const fwi_geom *geo, const float *v0, const float *dd, float *img)
{
    int rc = begin_call(c, g, geo);
    if (rc) return rc;
    const Plan &p = c->plan;
    if (!img) return set_err(c, FWI_EINVAL, "img is NULL");
    if (!dd && p.data_size > 0) return set_err(c, FWI_EINVAL, "dd is NULL");
    if ((rc = check_model(c, v0, "v0")) || (rc = prepare(c, v0))) return rc;
    if ((rc = ensure(c, c->samples, size_t(p.nt_max) * p.Q * 4))) return rc;
    TraceArgs t = trace_args(c);
    t.tr_in = dd;
    t.beta = 1.f;
    t.tm_out = static_cast<float *>(c->samples.p);
    if ((rc = other(c, launch_traces(t, c->stream, nullptr), "adjoint sources"))) return rc;
    Sweep w;
    if ((rc = forward_for_adjoint(c, v0, false, w))) return rc;
    if ((rc = backward_sweep(c, v0, w, img))) return rc;
    return finish_stats(c);
}

int fwi_rtm(fwi_ctx *c, const fwi_grid *g, const fwi_geom *geo, const float *v, const float *d_obs, float mute_v,
            float mute_pad, float mute_taper, float *img)
{
    int rc = begin_call(c, g, geo);
    if (rc) return rc;
    const Plan &p = c->plan;
    if (!img) return set_err(c, FWI_EINVAL, "img is NULL");
    if (!d_obs && p.data_size > 0) return set_err(c, FWI_EINVAL, "d_obs is NULL");
    if (!std::isfinite(mute_v) || !std::isfinite(mute_pad) || !std::isfinite(mute_taper) || mute_v < 0.f ||
        mute_taper < 0.f)
        return set_err(c, FWI_EINVAL, "mute: velocity and taper must be finite and >= 0 (velocity 0 = no mute)");
    if ((rc = check_model(c, v, "v")) || (rc = prepare(c, v))) return rc;
    const float *src = d_obs;
    if (mute_v > 0.f && p.data_size > 0) {
        // per-trace table: offset in the packed data, length, mute time
        HIPCHK(c, hipStreamSynchronize(c->stream));   // the previous table may still be in flight
        c->h_mute_off.clear();
        c->h_mute_nt.clear();
        c->h_mute_t0.clear();
        int64_t off = 0;
        for (int s = 0; s < geo->nshots; ++s) {
            const int32_t nt = geo->nt ? geo->nt[s] : g->nt_max;
            const double sz = geo->src_z[s] + (geo->src_fz ? geo->src_fz[s] : 0.f);
            const double sx = geo->src_x[s] + (geo->src_fx ? geo->src_fx[s] : 0.f);
            for (int64_t r = geo->rec_ptr[s]; r < geo->rec_ptr[s + 1]; ++r) {
                const double rz = geo->rec_z[r] + (geo->rec_fz ? geo->rec_fz[r] : 0.f);
                const double rx = geo->rec_x[r] + (geo->rec_fx ? geo->rec_fx[r] : 0.f);
                c->h_mute_off.push_back(off);
                c->h_mute_nt.push_back(nt);
                c->h_mute_t0.push_back(float(std::hypot(rz - sz, rx - sx) * g->h / mute_v + mute_pad));
                off += nt;
            }
        }
        if ((rc = upload(c, c->d_mute_off, c->h_mute_off)) || (rc = upload(c, c->d_mute_nt, c->h_mute_nt)) ||
            (rc = upload(c, c->d_mute_t0, c->h_mute_t0)) ||
            (rc = ensure(c, c->rtm_data, size_t(p.data_size) * 4)))
            return rc;
        if ((rc = other(c,
                        launch_mute(static_cast<const int64_t *>(c->d_mute_off.p),
                                    static_cast<const int32_t *>(c->d_mute_nt.p),
                                    static_cast<const float *>(c->d_mute_t0.p), int32_t(c->h_mute_t0.size()),
                                    g->dt, mute_taper, d_obs, static_cast<float *>(c->rtm_data.p), c->stream),
                        "mute")))
            return rc;
        src = static_cast<const float *>(c->rtm_data.p);
    }
    if ((rc = ensure(c, c->samples, size_t(p.nt_max) * p.Q * 4)) ||
        (rc = ensure(c, c->rtm_img, size_t(g->nz) * g->nx * 4)))
        return rc;
    TraceArgs t = trace_args(c);
    t.tr_in = src;
    t.beta = 1.f;
    t.tm_out = static_cast<float *>(c->samples.p);
    if ((rc = other(c, launch_traces(t, c->stream, nullptr), "adjoint sources"))) return rc;
    Sweep w;
    if ((rc = forward_for_adjoint(c, v, false, w))) return rc;
    float *mig = static_cast<float *>(c->rtm_img.p);
    if ((rc = backward_sweep(c, v, w, mig))) return rc;
    if ((rc = other(c, launch_laplace5(mig, g->nz, g->nx, img, c->stream), "laplacian"))) return rc;
    return finish_stats(c);
}

}  // extern "C"
