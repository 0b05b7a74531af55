// Driver of the host kernel emulation: runs every public entry point of the
// library through the C ABI on a geometry read from a text file, for a list
// of tilings (or the autotuner), and the deblurring network for one
// configuration. Any out-of-bounds kernel access aborts the process with an
// AddressSanitizer report.
//
//   emu_driver fd  <geom> <spec>...      spec: "auto" or "cw,rows,levels,prefetch,ckpt_every"
//   emu_driver net <depth> <base> <H> <W> <nz> <nx>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "deblur.h"
#include "fwi.h"

void emu_print_launches();

static fwi_ctx *g_ctx = nullptr;
static deblur_net *g_net = nullptr;

#define CK(call)                                                                                 \
    do {                                                                                         \
        int rc_ = (call);                                                                        \
        if (rc_) {                                                                               \
            std::fprintf(stderr, "FAIL %s rc=%d: %s\n", #call, rc_, fwi_last_error(g_ctx));     \
            std::exit(1);                                                                        \
        }                                                                                        \
    } while (0)
#define DK(call)                                                                                 \
    do {                                                                                         \
        int rc_ = (call);                                                                        \
        if (rc_) {                                                                               \
            std::fprintf(stderr, "FAIL %s rc=%d: %s\n", #call, rc_, deblur_last_error(g_net));  \
            std::exit(1);                                                                        \
        }                                                                                        \
    } while (0)

template <class T>
static T *dev(size_t n)
{
    return static_cast<T *>(std::calloc(n ? n : 1, sizeof(T)));
}

static int run_fd(int argc, char **argv)
{
    const char *path = argv[2];
    FILE *f = std::fopen(path, "r");
    if (!f) return 2;
    fwi_grid g{};
    int S = 0, has_win = 0, has_nt = 0, shared = 1, has_frac = 0;
    if (std::fscanf(f, "%d %d %d %f %f %d %f %f %d %d %d %d %d %d %d", &g.nz, &g.nx, &g.nb, &g.h, &g.dt, &g.nt_max,
                    &g.v_ref, &g.R, &S, &has_win, &has_nt, &shared, &has_frac, &g.free_surface, &g.pml) != 15)
        return 2;
    std::vector<int32_t> sz(S), sx(S), wx0(S), wnx(S), nt(S), rz, rx;
    std::vector<float> sfz(S), sfx(S), rfz, rfx;
    std::vector<int64_t> rptr(1, 0);
    for (int s = 0; s < S; ++s) {
        int nr = 0;
        if (std::fscanf(f, "%d %d %d %d %d %d %f %f", &sz[s], &sx[s], &wx0[s], &wnx[s], &nt[s], &nr, &sfz[s],
                        &sfx[s]) != 8)
            return 2;
        for (int i = 0; i < nr; ++i) {
            int z, x;
            float fz, fx;
            if (std::fscanf(f, "%d %d %f %f", &z, &x, &fz, &fx) != 4) return 2;
            rz.push_back(z);
            rx.push_back(x);
            rfz.push_back(fz);
            rfx.push_back(fx);
        }
        rptr.push_back(rptr.back() + nr);
    }
    std::vector<float> wav(size_t(shared ? 1 : S) * g.nt_max);
    for (auto &w : wav)
        if (std::fscanf(f, "%f", &w) != 1) return 2;
    const size_t nm = size_t(g.nz) * g.nx;
    std::vector<float> hv0(nm), hvt(nm);
    for (auto &v : hv0)
        if (std::fscanf(f, "%f", &v) != 1) return 2;
    for (auto &v : hvt)
        if (std::fscanf(f, "%f", &v) != 1) return 2;
    std::fclose(f);
    fwi_geom geo{};
    geo.nshots = S;
    geo.src_z = sz.data();
    geo.src_x = sx.data();
    geo.win_x0 = has_win ? wx0.data() : nullptr;
    geo.win_nx = has_win ? wnx.data() : nullptr;
    geo.nt = has_nt ? nt.data() : nullptr;
    geo.rec_ptr = rptr.data();
    geo.rec_z = rz.data();
    geo.rec_x = rx.data();
    geo.wavelet = wav.data();
    geo.wavelet_shared = shared;
    if (has_frac) {
        geo.src_fz = sfz.data();
        geo.src_fx = sfx.data();
        geo.rec_fz = rfz.data();
        geo.rec_fx = rfx.data();
    }
    int64_t ndata = 0;
    for (int s = 0; s < S; ++s) ndata += (rptr[s + 1] - rptr[s]) * (has_nt ? nt[s] : g.nt_max);

    for (int a = 3; a < argc; ++a) {
        fwi_ctx *c = nullptr;
        if (fwi_ctx_create(0, nullptr, &c)) return 3;
        g_ctx = c;
        CK(fwi_ctx_set_graphs(c, 0));
        const std::string spec = argv[a];
        int cw = 0, rows = 0, tb = 0, pd = 0, ck = 0, slots = -1;
        if (spec != "auto") {
            const int nf = std::sscanf(spec.c_str(), "%d,%d,%d,%d,%d,%d", &cw, &rows, &tb, &pd, &ck, &slots);
            if (nf != 5 && nf != 6) return 2;
            CK(fwi_ctx_set_tiling(c, -1, cw, rows, tb, pd));
            CK(fwi_ctx_set_ckpt_slots(c, slots));
            // optional tilings of single kernel classes: EMU_TILING_<class>="cw,rows,levels,prefetch"
            for (int k = 0; k < 4; ++k) {
                char name[32];
                std::snprintf(name, sizeof name, "EMU_TILING_%d", k);
                if (const char *e = std::getenv(name)) {
                    int t[4] = {0, 0, 0, 0};
                    if (std::sscanf(e, "%d,%d,%d,%d", &t[0], &t[1], &t[2], &t[3]) == 4)
                        CK(fwi_ctx_set_tiling(c, k, t[0], t[1], t[2], t[3]));
                }
            }
        }
        g.ckpt_every = ck;
        float *v0 = dev<float>(nm), *vt = dev<float>(nm), *grad = dev<float>(nm), *img = dev<float>(nm);
        float *grad2 = dev<float>(nm), *img2 = dev<float>(nm), *img3 = dev<float>(nm), *img4 = dev<float>(nm);
        float *dobs = dev<float>(size_t(ndata)), *dd = dev<float>(size_t(ndata)), *dsyn = dev<float>(size_t(ndata));
        std::memcpy(v0, hv0.data(), nm * 4);
        std::memcpy(vt, hvt.data(), nm * 4);
        double phi = 0;
        CK(fwi_forward(c, &g, &geo, vt, dobs));
        // the allocation-free forward: the same bits from the static scratch
        CK(fwi_forward_noalloc(c, &g, &geo, vt, dd));
        if (ndata > 0 && std::memcmp(dd, dobs, size_t(ndata) * 4) != 0) {
            std::fprintf(stderr, "FAIL fwi_forward_noalloc differs from fwi_forward (%s)\n", spec.c_str());
            std::exit(1);
        }
        CK(fwi_gradient_pair(c, &g, &geo, v0, dobs, grad, &phi, -1.f, img4, dd));
        CK(fwi_gradient(c, &g, &geo, v0, dobs, grad2, &phi, dsyn));
        CK(born_pair(c, &g, &geo, v0, grad, dd, img3));
        CK(born_demig(c, &g, &geo, v0, grad, dd));
        CK(born_mig(c, &g, &geo, v0, dd, img2));
        CK(fwi_rtm(c, &g, &geo, v0, dobs, 1500.f, 0.01f, 0.02f, img));
        fwi_stats st{};
        fwi_ctx_get_stats(c, &st);
        CK(fwi_misfit(c, &g, &geo, v0, dobs, &phi));
        // FNV-1a over the bits of the gradients and the images (migration,
        // born_pair, the fused gradient + pair): the same for every tiling
        // and checkpointing schedule
        auto fnv = [&](const float *q) {
            uint64_t h = 1469598103934665603ULL;
            for (size_t i = 0; i < nm; ++i) {
                uint32_t b;
                std::memcpy(&b, q + i, 4);
                for (int byte = 0; byte < 4; ++byte) h = (h ^ ((b >> (8 * byte)) & 0xffu)) * 1099511628211ULL;
            }
            return (unsigned long long)h;
        };
        std::printf("ok %s tile_fwd=%d,%d,%d,%d segments=%d slots=%d recomputed=%lld "
                    "hash=%016llx,%016llx,%016llx,%016llx,%016llx\n",
                    spec.c_str(), st.tile_cw[0], st.tile_rows[0], st.tile_levels[0], st.tile_prefetch[0],
                    st.n_segments, st.ckpt_slots, (long long)st.recomputed_steps, fnv(grad), fnv(grad2), fnv(img2),
                    fnv(img3), fnv(img4));
        std::fflush(stdout);
        for (float *p : {v0, vt, grad, img, grad2, img2, img3, img4, dobs, dd, dsyn}) std::free(p);
        fwi_ctx_destroy(c);
        g_ctx = nullptr;
    }
    return 0;
}

static int run_net(int argc, char **argv)
{
    if (argc < 8) return 2;
    deblur_cfg cfg{std::atoi(argv[2]), std::atoi(argv[3]), 0.2f, std::atoi(argv[4]), std::atoi(argv[5])};
    const int nz = std::atoi(argv[6]), nx = std::atoi(argv[7]);
    fwi_ctx *c = nullptr;
    if (fwi_ctx_create(0, nullptr, &c)) return 3;
    g_ctx = c;
    if (deblur_create(c, &cfg, 7, &g_net)) return 4;
    const size_t n = size_t(nz) * nx, P = size_t(cfg.in_h) * cfg.in_w;
    float *x = dev<float>(n), *y = dev<float>(n), *q = dev<float>(n);
    float *xr = dev<float>(P), *tr = dev<float>(P), *yr = dev<float>(P);
    uint64_t s = 12345;
    auto rnd = [&]() {
        s = s * 6364136223846793005ULL + 1442695040888963407ULL;
        return float(int64_t(s >> 33) % 2001 - 1000) * 1e-3f;
    };
    for (size_t i = 0; i < n; ++i) {
        x[i] = rnd();
        y[i] = rnd();
    }
    for (size_t i = 0; i < P; ++i) {
        xr[i] = rnd();
        tr[i] = rnd();
    }
    float hist[2];
    DK(deblur_train(c, g_net, x, y, nz, nx, 1, 1e-3f, hist));
    DK(deblur_apply(c, g_net, x, nz, nx, q));
    DK(deblur_forward_raw(c, g_net, xr, yr));
    int64_t np = 0;
    DK(deblur_num_params(g_net, &np));
    std::vector<float> grads(static_cast<size_t>(np));
    double loss = 0;
    DK(deblur_grad_raw(c, g_net, xr, tr, &loss, grads.data()));
    std::printf("ok net depth=%d base=%d %dx%d\n", cfg.depth, cfg.base_ch, cfg.in_h, cfg.in_w);
    deblur_destroy(g_net);
    fwi_ctx_destroy(c);
    for (float *p : {x, y, q, xr, tr, yr}) std::free(p);
    return 0;
}

int main(int argc, char **argv)
{
    if (argc < 2) return 2;
    const std::string what = argv[1];
    const int rc = what == "fd" ? run_fd(argc, argv) : what == "net" ? run_net(argc, argv) : 2;
    if (rc == 0) emu_print_launches();
    return rc;
}
