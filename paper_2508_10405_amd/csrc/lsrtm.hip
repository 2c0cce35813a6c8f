// Runtime of the LSRTM library: context, memory plan, passes, CGNR.
//
// Pass structure (one launch group = a contiguous range of shots advanced by
// the same kernel launches):
//   forward : background steps, p recorded at the receivers, background
//             checkpoints stored every k steps.
//   born    : background + scattered steps (section 2, eq. scattereqln),
//             scattered pressure recorded (section 3, L dm := R du).
//   adjoint : for each checkpoint segment, last first: restore the background
//             state, replay k steps storing G_a p + psi_a (the gradient behind
//             dv_a) and q, then run the k adjoint steps backwards, on the
//             scaled state Q = -dt kappa p~, U_a = -dt b_a v~_a, with the
//             imaging conditions (appendix A,
//             eqs. gradlsm, gradrho, gradkappa).  The images of every shot
//             are added in shot order into an FP64 accumulator and mapped to
//             (lnVp, lnIp) by the chain rule of section 3.
// Checkpoints do not depend on the perturbation, so they are stored once per
// model and acquisition and reused by every later pass; for the same reason
// the replays of the last segments of every launch group may be kept in HBM
// the memory plan leaves over (the replay cache) and read by every later
// migration pass instead of being recomputed, and by every later 2D Born pass
// in place of the background steps of those segments.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lsrtm.h"
#include "kernels.h"

using namespace lsrtm;

namespace {

// Exact O(2,8) staggered weights c_k (odd-moment conditions at half offsets).
const double kC8[4] = {1225.0 / 1024.0, -245.0 / 3072.0, 49.0 / 5120.0, -5.0 / 7168.0};

struct Window {
    int lo[3], hi[3];
    int N[3];
    int ldz;
    long long sx, sy, npts;
    float* kdt = nullptr;
    float* sb = nullptr;
    float* bdt[3] = {nullptr, nullptr, nullptr};
    float* dlnr = nullptr;
    float* dlnk = nullptr;
    float* cpml[3] = {nullptr, nullptr, nullptr};
};

struct ShotInfo {
    int win;
    int src_lin;
    int rec0, nrec;
    long long data_off;
    long long ckbytes;
    std::vector<int> rec_lin;
};

struct Group {
    int s0 = 0, ns = 0;
    std::vector<Slot> h_slots;
    Slot* d_slots = nullptr;       // descriptors (fused schedule: even steps)
    Slot* d_alt = nullptr;         // fused schedule: roles of the two buffers swapped
    int4* d_tiles = nullptr;
    int ntiles = 0;
    int tiles_for = -1;            // tile id the table was built for
    Rec* d_rec = nullptr;
    int nrec = 0;
    int* d_node_slot = nullptr;
    int* d_node_idx = nullptr;
    int* d_node_ptr = nullptr;
    Rec* d_node_rec = nullptr;
    int nnode = 0;
    int* d_win = nullptr;
    int* d_trp = nullptr;          // 2D: receivers per tile (CSR over the tile table)
    Rec* d_trec = nullptr;
    // tables of other tile shapes for the phases without receivers
    struct AltTiles {
        int tile;
        int4* d;
        int n;
    };
    std::vector<AltTiles> alt;
    std::vector<Rec> h_rec;        // receivers of the group (host copy)
    // replay cache: descriptors of the cached segments ([rc_m][ns], equal to
    // d_slots but for seg), and whether the cache holds this group's replays
    Slot* d_rc = nullptr;
    bool rc_valid = false;
    long long max_npts = 0;
    long long bg_used = 0, sc_used = 0, img_used = 0;   // floats
};

struct EvPair {
    hipEvent_t a, b;
    int cls;
};

}  // namespace

struct lsrtm_ctx {
    lsrtm_grid g{};
    hipStream_t st = nullptr;
    std::string err;
    Coef C{};
    int ndim = 2;
    // model
    float* lnvp = nullptr;
    float* lnip = nullptr;
    long long gpts = 0;
    double vmax = 0.0;
    bool have_model = false;
    // acquisition
    int nshot = 0;
    bool have_acq = false;
    std::vector<ShotInfo> shots;
    std::vector<Window> wins;
    std::vector<int> h_win;        // [nshot][6]
    float* src_amp = nullptr;      // [nshot][nt]
    long long data_len = 0;
    long long padded_total = 0;
    // plan
    int G = 1, k = 1, nseg = 1, S = 1;
    int tile = -1;
    long long plan_bytes = 0;
    std::vector<Group> groups;
    long long bg_region = 0, sc_region = 0, img_region = 0;
    float* pool = nullptr;
    float* segbuf = nullptr;
    float* rcache = nullptr;       // replay cache: the last rc_m segments of every group
    int rc_m = 0;
    char* ckbuf = nullptr;
    float* ckscales = nullptr;     // [nseg][nshot][1+ndim]
    float* partial = nullptr;      // reduction workspace of set_model
    float* ckpart = nullptr;       // checkpoint max-abs partials [G][1+ndim][nblk]
    int nblk = 64;                 // blocks per field of the max-abs pass (set by the plan)
    double* dpart = nullptr;
    double* dscal = nullptr;       // device scalar results
    int* d_flag = nullptr;
    double* acc64 = nullptr;       // [2][gpts]
    bool ckpt_valid = false;
    bool ck_group = false;         // checkpoints held for the active group only
    bool fused = false;            // 2D one-kernel-per-step schedule
    // CG workspace
    float* cg_r = nullptr;
    float* cg_w = nullptr;
    float* cg_z = nullptr;
    float* cg_p = nullptr;
    double cg_zz = 0.0, cg_r0 = 0.0, cg_rr = 0.0;   // cg_zz = <z, s> (= <z, z> unpreconditioned)
    double cg_alpha = 0.0, cg_beta = 0.0, cg_ww = 0.0;   // step of the last iteration
    int cg_k = 0;
    bool cg_active = false;
    // diagonal preconditioner M^-1 of the normal residual (pseudo-Hessian)
    float* cg_minv = nullptr;      // [2][gpts], library copy
    float* cg_s = nullptr;         // normal residual L^T r when preconditioned
    bool precond = false;          // a preconditioner is set
    bool cg_pre = false;           // the current CG run is preconditioned
    // PSF Hessian (image domain)
    int* psf_tab = nullptr;        // corner/weight tables of psf_spacing
    int psf_spacing = 0;
    float* psf_dm = nullptr;       // [2][gpts] scatterer model
    float* psf_d = nullptr;        // data of the scatterer model
    float* psf_v[4] = {nullptr, nullptr, nullptr, nullptr};   // image-domain CG: r, z, p, w
    WienerWork* wiener = nullptr;  // FFT plans and buffers of the Wiener filter
    // options
    int opt_spl = 0;
    int opt_tile = -1;
    int opt_graph = 1;
    int opt_timing = 0;
    long long opt_budget_mb = 0;
    int opt_ckg = 0;
    int opt_fused = 0;
    int opt_progress = 0;
    int opt_tile_v = -1;           // two-phase steps: tile of the velocity phases (-1: tile)
    int opt_tile_a = -1;           // two-phase steps: tile of the adjoint A phase (-1: tile)
    long long opt_rcache_mb = 0;   // HBM the replay cache may take (0: none)
    // timing
    std::vector<EvPair> evpool;
    size_t evused = 0;
    int tstride = 16;              // time the launches of every tstride-th step
    bool tnow = true;              // the current step is timed
    bool tpending = false;
    double kms[LSRTM_NKERNEL] = {0};
    long long kcnt[LSRTM_NKERNEL] = {0};
    double pass_ms = 0.0;
    hipEvent_t pa = nullptr, pb = nullptr;
    // acquisition inputs (kept so that the plan can be rebuilt)
    std::vector<int> a_win, a_src, a_recptr, a_rec;
    float* wavelet = nullptr;      // device copy [nshot][nt]
    // HIP graphs of whole passes, per launch group, least recently used
    // first in graph_lru; at most graph_cap of them are kept
    std::map<std::tuple<int, int, const void*, int>, hipGraphExec_t> graphs;
    std::list<std::tuple<int, int, const void*, int>> graph_lru;
    size_t graph_cap = 0;
    hipStream_t gst = nullptr;     // capture/replay stream (default priority)
    hipEvent_t gin = nullptr, gout = nullptr;
    bool tuned = false;
    // allocations
    std::vector<void*> allocs;
    std::vector<void*> acq_allocs;
};

namespace {

#define FAIL(ctx, code, ...)                                                     \
    do {                                                                         \
        char _b[512];                                                            \
        snprintf(_b, sizeof(_b), __VA_ARGS__);                                   \
        (ctx)->err = _b;                                                         \
        return (code);                                                           \
    } while (0)

#define HIPCHK(ctx, call)                                                        \
    do {                                                                         \
        hipError_t _e = (call);                                                  \
        if (_e != hipSuccess)                                                    \
            FAIL(ctx, LSRTM_EHIP, "%s: %s (%s:%d)", #call, hipGetErrorString(_e), \
                 __FILE__, __LINE__);                                            \
    } while (0)

#define CHK(call)                                                                \
    do {                                                                         \
        lsrtm_status _s = (call);                                                \
        if (_s != LSRTM_OK) return _s;                                           \
    } while (0)

lsrtm_status dalloc(lsrtm_ctx* c, void** p, size_t bytes, bool acq) {
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        FAIL(c, LSRTM_ENOMEM, "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    (acq ? c->acq_allocs : c->allocs).push_back(*p);
    return LSRTM_OK;
}

template <typename T>
lsrtm_status dalloc_t(lsrtm_ctx* c, T** p, size_t n, bool acq) {
    return dalloc(c, reinterpret_cast<void**>(p), n * sizeof(T), acq);
}

// The background changed (model, or a failed snapshot): stored checkpoints
// and cached replays are stale.
void background_changed(lsrtm_ctx* c) {
    c->ckpt_valid = false;
    for (auto& gr : c->groups) gr.rc_valid = false;
}

void clear_graphs(lsrtm_ctx* c) {
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    c->graph_lru.clear();
}

void free_acq(lsrtm_ctx* c) {
    clear_graphs(c);
    for (void* p : c->acq_allocs) (void)hipFree(p);
    c->acq_allocs.clear();
    c->groups.clear();
    c->wins.clear();
    c->shots.clear();
    c->have_acq = false;
    c->ckpt_valid = false;
    c->pool = nullptr;
    c->segbuf = nullptr;
    c->rcache = nullptr;
    c->rc_m = 0;
    c->ckbuf = nullptr;
    c->ckscales = nullptr;
    c->ckpart = nullptr;
    c->acc64 = nullptr;
    c->cg_r = c->cg_w = c->cg_z = c->cg_p = nullptr;
    c->psf_d = nullptr;
    c->cg_active = false;
    c->src_amp = nullptr;
}

long long round_up(long long a, long long m) { return (a + m - 1) / m * m; }

// Consecutive launch groups of at most G shots, sizes balanced to within one.
std::vector<int> group_sizes(int nshot, int G) {
    const int ng = (nshot + G - 1) / G;
    std::vector<int> v(ng, nshot / ng);
    for (int i = 0; i < nshot % ng; ++i) v[i] += 1;
    return v;
}

// 1D CPML coefficients along one padded axis of N nodes.
void cpml_axis(int N, int npml, double h, double dt, double vmax, double R, double f0, bool half,
               std::vector<float>& ac, std::vector<float>& bc) {
    ac.assign(N, 0.f);
    bc.assign(N, 1.f);
    if (npml <= 0) return;
    const double first = npml, last = N - npml - 1;
    const double d0 = -3.0 * vmax * std::log(R) / (2.0 * npml * h);
    for (int i = 0; i < N; ++i) {
        const double pos = i + (half ? 0.5 : 0.0);
        const double dist = pos < first ? first - pos : (pos > last ? pos - last : 0.0);
        const double xi = std::min(1.0, dist / npml);
        const double d = d0 * xi * xi;
        const double alpha = M_PI * f0 * (1.0 - xi);
        const double b = std::exp(-(d + alpha) * dt);
        ac[i] = d > 0.0 ? (float)(d * (b - 1.0) / (d + alpha)) : 0.f;
        bc[i] = (float)b;
    }
}

int strip_depth(const lsrtm_ctx* c) { return c->g.npml + 1; }

long long strip_count_h(const int N[3], int a, int Sd) {
    const int Sa = std::min(Sd, N[a]);
    long long cnt = 2LL * Sa;
    for (int b = 0; b < 3; ++b)
        if (b != a) cnt *= N[b];
    return cnt;
}

// ---------------------------------------------------------------------------
// Timing
// ---------------------------------------------------------------------------
// The next free event pair for a sample of class cls, or null when this step
// is not sampled.
EvPair* tpick(lsrtm_ctx* c, int cls) {
    if (!c->opt_timing || !c->tnow) return nullptr;
    if (c->evused == c->evpool.size()) {
        EvPair e;
        if (hipEventCreate(&e.a) != hipSuccess || hipEventCreate(&e.b) != hipSuccess) {
            c->opt_timing = 0;
            return nullptr;
        }
        c->evpool.push_back(e);
    }
    EvPair& e = c->evpool[c->evused];
    e.cls = cls;
    return &e;
}

// Time a group of launches between two event records (checkpoints, receivers).
void tbeg(lsrtm_ctx* c, int cls) {
    c->tpending = false;
    EvPair* e = tpick(c, cls);
    if (!e) return;
    (void)hipEventRecord(e->a, c->st);
    c->tpending = true;
}

void tend(lsrtm_ctx* c) {
    if (!c->tpending) return;
    (void)hipEventRecord(c->evpool[c->evused].b, c->st);
    c->evused++;
    c->tpending = false;
}

void tstep(lsrtm_ctx* c, int n) { c->tnow = (n % c->tstride) == 0; }

lsrtm_status pass_begin(lsrtm_ctx* c) {
    for (int i = 0; i < LSRTM_NKERNEL; ++i) {
        c->kms[i] = 0.0;
        c->kcnt[i] = 0;
    }
    c->evused = 0;
    if (!c->pa) {
        HIPCHK(c, hipEventCreate(&c->pa));
        HIPCHK(c, hipEventCreate(&c->pb));
    }
    HIPCHK(c, hipEventRecord(c->pa, c->st));
    return LSRTM_OK;
}

lsrtm_status pass_end(lsrtm_ctx* c) {
    HIPCHK(c, hipEventRecord(c->pb, c->st));
    HIPCHK(c, hipEventSynchronize(c->pb));
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->pa, c->pb));
    c->pass_ms = ms;
    for (size_t i = 0; i < c->evused; ++i) {
        float t = 0.f;
        HIPCHK(c, hipEventElapsedTime(&t, c->evpool[i].a, c->evpool[i].b));
        c->kms[c->evpool[i].cls] += t;
        c->kcnt[c->evpool[i].cls] += 1;
    }
    c->evused = 0;
    return LSRTM_OK;
}

// ---------------------------------------------------------------------------
// Tiles
// ---------------------------------------------------------------------------
int default_tile(int ndim) { return ndim == 2 ? 1 : 1; }

void tile_shape(int ndim, int id, int* bz, int* bx, int* by) {
    if (ndim == 2) {
        *bz = kTiles2[id][0];
        *bx = kTiles2[id][1];
        *by = 1;
    } else {
        *bz = kTiles3[id][0];
        *bx = kTiles3[id][1];
        *by = kTiles3[id][2];
    }
}

// Tile table of a group: (slot, z0, x0, w) of every tile of every slot; in
// 3D w = y0 | y1 << 16, the planes y0 .. y1 - 1 of the tile's march.
void tile_list(const lsrtm_ctx* c, const Group& gr, int tile, std::vector<int4>& t) {
    int bz, bx, by;
    tile_shape(c->ndim, tile, &bz, &bx, &by);
    t.clear();
    for (int s = 0; s < gr.ns; ++s) {
        const Slot& S = gr.h_slots[s];
        for (int y0 = 0; y0 < S.n[2]; y0 += by) {
            const int y1 = std::min(y0 + by, S.n[2]);
            for (int x0 = 0; x0 < S.n[1]; x0 += bx)
                for (int z0 = 0; z0 < S.n[0]; z0 += bz)
                    t.push_back(make_int4(s, z0, x0, c->ndim == 3 ? y0 | (y1 << 16) : 0));
        }
    }
}

// Tables of the receiver-free phases' own tile shapes (two-phase steps).
lsrtm_status build_alt_tiles(lsrtm_ctx* c, Group& gr) {
    if (c->fused) return LSRTM_OK;
    for (int tile : {c->opt_tile_v, c->opt_tile_a}) {
        if (tile < 0) continue;
        bool have = false;
        for (const auto& a : gr.alt) have = have || a.tile == tile;
        if (have) continue;
        std::vector<int4> t;
        tile_list(c, gr, tile, t);
        Group::AltTiles a{tile, nullptr, (int)t.size()};
        CHK(dalloc_t(c, &a.d, t.size(), true));
        HIPCHK(c, hipMemcpy(a.d, t.data(), t.size() * sizeof(int4), hipMemcpyHostToDevice));
        gr.alt.push_back(a);
    }
    return LSRTM_OK;
}

lsrtm_status build_tiles(lsrtm_ctx* c, Group& gr, int tile) {
    CHK(build_alt_tiles(c, gr));
    if (gr.tiles_for == tile) return LSRTM_OK;
    int bz, bx, by;
    tile_shape(c->ndim, tile, &bz, &bx, &by);
    std::vector<int4> t;
    tile_list(c, gr, tile, t);
    if (gr.d_tiles) {
        (void)hipFree(gr.d_tiles);
        auto it = std::find(c->acq_allocs.begin(), c->acq_allocs.end(), (void*)gr.d_tiles);
        if (it != c->acq_allocs.end()) c->acq_allocs.erase(it);
        gr.d_tiles = nullptr;
    }
    CHK(dalloc_t(c, &gr.d_tiles, t.size(), true));
    HIPCHK(c, hipMemcpy(gr.d_tiles, t.data(), t.size() * sizeof(int4), hipMemcpyHostToDevice));
    gr.ntiles = (int)t.size();
    gr.tiles_for = tile;
    if (c->ndim == 2) {
        // receivers by tile: tile of node (z, x) of slot s and its tile-local index
        std::vector<long long> base(gr.ns + 1, 0);
        for (int s = 0; s < gr.ns; ++s) {
            const Slot& S = gr.h_slots[s];
            base[s + 1] = base[s] + (long long)((S.n[0] + bz - 1) / bz) * ((S.n[1] + bx - 1) / bx);
        }
        std::vector<std::vector<Rec>> per(gr.ntiles);
        for (const Rec& R : gr.h_rec) {
            const Slot& S = gr.h_slots[R.slot];
            const int z = R.idx % S.ldz, x = R.idx / S.ldz;
            const int ntz = (S.n[0] + bz - 1) / bz;
            const long long ti = base[R.slot] + (long long)(x / bx) * ntz + z / bz;
            Rec T = R;
            T.idx = (z % bz) + bz * (x % bx);
            per[ti].push_back(T);
        }
        std::vector<int> ptr(gr.ntiles + 1, 0);
        std::vector<Rec> all;
        for (int i = 0; i < gr.ntiles; ++i) {
            all.insert(all.end(), per[i].begin(), per[i].end());
            ptr[i + 1] = (int)all.size();
        }
        for (void** pp : {(void**)&gr.d_trp, (void**)&gr.d_trec}) {
            if (*pp) {
                (void)hipFree(*pp);
                auto it = std::find(c->acq_allocs.begin(), c->acq_allocs.end(), *pp);
                if (it != c->acq_allocs.end()) c->acq_allocs.erase(it);
                *pp = nullptr;
            }
        }
        CHK(dalloc_t(c, &gr.d_trp, ptr.size(), true));
        CHK(dalloc_t(c, &gr.d_trec, std::max<size_t>(1, all.size()), true));
        HIPCHK(c, hipMemcpy(gr.d_trp, ptr.data(), ptr.size() * sizeof(int), hipMemcpyHostToDevice));
        if (!all.empty())
            HIPCHK(c, hipMemcpy(gr.d_trec, all.data(), all.size() * sizeof(Rec), hipMemcpyHostToDevice));
    }
    return LSRTM_OK;
}

const Slot* desc(const Group& gr, int par) { return ((par & 1) && gr.d_alt) ? gr.d_alt : gr.d_slots; }

lsrtm_status stencil(lsrtm_ctx* c, Group& gr, int kind, int n, int sstep, int flag, const Slot* sl,
                     TileRec tr = TileRec{nullptr, nullptr, nullptr, nullptr}) {
    static const int cls_of[8] = {2, 3, 2, 3, 0, 1, 4, 5};
    // a sampled launch carries its own start / end events; the Born phases on
    // a cached background move fewer bytes and are not sampled, so that the
    // per-kernel figures stay those of one kernel
    const bool rc = kind == K_BORN_V_RC || kind == K_BORN_P_RC;
    EvPair* ev = rc ? nullptr : tpick(c, cls_of[kind]);
    hipEvent_t e0 = ev ? ev->a : nullptr, e1 = ev ? ev->b : nullptr;
    hipError_t e;
    if (c->fused) e = launch2f(kind, c->tile, gr.ntiles, c->st, sl, gr.d_tiles, c->C, n, sstep, flag, tr, e0, e1);
    else {
        // the velocity phases and the adjoint A phase touch no receivers (in
        // 3D none of the phases does; the 2D P and B phases use the stencil
        // tile's receiver lists) and may walk a table of their own tile shape
        const bool vph = kind == K_BG_V || kind == K_SEG_V || kind == K_BORN_V || kind == K_BORN_V_RC;
        const int want = vph ? c->opt_tile_v : kind == K_ADJ_A ? c->opt_tile_a : -1;
        int tile = c->tile, nt = gr.ntiles;
        const int4* tab = gr.d_tiles;
        if (want >= 0 && want != c->tile) {
            for (const auto& a : gr.alt)
                if (a.tile == want) {
                    tile = a.tile;
                    nt = a.n;
                    tab = a.d;
                }
            if (tab == gr.d_tiles) FAIL(c, LSRTM_ESTATE, "tile table %d of phase %d was not built", want, kind);
        }
        if (c->ndim == 3) e = launch3d(kind, tile, nt, c->st, sl, tab, c->C, n, sstep, flag, e0, e1);
        else e = launch2d(kind, tile, nt, c->st, sl, tab, c->C, n, sstep, flag, tr, e0, e1);
    }
    if (e != hipSuccess) FAIL(c, LSRTM_EHIP, "stencil launch (kind %d): %s", kind, hipGetErrorString(e));
    if (ev) c->evused++;
    return LSRTM_OK;
}

lsrtm_status ckpt(lsrtm_ctx* c, Group& gr, int j, bool save, const Slot* sl) {
    CkptArgs a;
    a.slots = sl;
    a.nslot = gr.ns;
    a.ndim = c->ndim;
    a.dtype = c->g.ckpt_dtype;
    a.S = c->S;
    a.j = j;
    a.scales = c->ckscales + ((long long)j * c->nshot + gr.s0) * (1 + c->ndim);
    a.partial = c->ckpart;
    a.nblk = c->nblk;
    a.nonfinite = c->d_flag;
    tbeg(c, 6);
    hipError_t e = save ? launch_ckpt_save(a, gr.max_npts, c->st) : launch_ckpt_load(a, gr.max_npts, c->st);
    tend(c);
    if (e != hipSuccess) FAIL(c, LSRTM_EHIP, "checkpoint kernel: %s", hipGetErrorString(e));
    return LSRTM_OK;
}

lsrtm_status fill(lsrtm_ctx* c, float* p, long long n) {
    HIPCHK(c, launch_fill(p, n, 0.f, c->st));
    return LSRTM_OK;
}

lsrtm_status check_flag(lsrtm_ctx* c) {
    int f = 0;
    HIPCHK(c, hipMemcpyAsync(&f, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (f) {
        background_changed(c);
        HIPCHK(c, launch_fill(reinterpret_cast<float*>(c->d_flag), 1, 0.f, c->st));
        FAIL(c, LSRTM_ENONFINITE, "non-finite value in a stored background snapshot");
    }
    return LSRTM_OK;
}

// ---------------------------------------------------------------------------
// Passes of one launch group
// ---------------------------------------------------------------------------
// mode 0: forward (record p), 1: born (record dp), 2: forward without data.
// With the fused schedule the step reads the buffers of parity n % 2 and
// writes the other ones.
lsrtm_status group_forward(lsrtm_ctx* c, Group& gr, int mode, float* d, bool write_ck) {
    CHK(build_tiles(c, gr, c->tile));
    CHK(fill(c, c->pool, gr.bg_used));
    if (mode == 1) CHK(fill(c, c->pool + c->bg_region, gr.sc_used));
    const bool fz = c->fused;
    // 2D Born steps inside the segments whose replays the cache holds read
    // the background from there instead of advancing it (nothing after them
    // needs the background state)
    const int jc = c->nseg - c->rc_m;
    const bool use_rc = mode == 1 && !write_ck && c->rc_m > 0 && gr.rc_valid && c->ndim == 2 && !fz;
    for (int n = 0; n < c->g.nt; ++n) {
        tstep(c, n);
        const int j = n / c->k;
        const bool rcs = use_rc && j >= jc;
        const Slot* cur = rcs ? gr.d_rc + (long long)(j - jc) * gr.ns : desc(gr, fz ? n : 0);
        if (write_ck && n > 0 && n % c->k == 0) CHK(ckpt(c, gr, n / c->k, true, cur));
        const int kv = rcs ? K_BORN_V_RC : mode == 1 ? K_BORN_V : K_BG_V;
        const int kp = rcs ? K_BORN_P_RC : mode == 1 ? K_BORN_P : K_BG_P;
        const int sstep = rcs ? n - j * c->k : 0;
        // 2D kernels record the receivers themselves
        const TileRec tr{gr.d_trp, gr.d_trec, mode != 2 ? d : nullptr, nullptr};
        const TileRec none{nullptr, nullptr, nullptr, nullptr};
        CHK(stencil(c, gr, kv, n, sstep, 0, cur, fz ? tr : none));
        if (!fz) CHK(stencil(c, gr, kp, n, sstep, 0, cur, tr));
        if (mode != 2 && c->ndim == 3) {
            tbeg(c, 7);
            hipError_t e = launch_gather(desc(gr, fz ? n + 1 : 0), gr.d_rec, gr.nrec, n, mode == 1, d, c->st);
            tend(c);
            if (e != hipSuccess) FAIL(c, LSRTM_EHIP, "gather: %s", hipGetErrorString(e));
        }
    }
    return LSRTM_OK;
}

lsrtm_status group_adjoint(lsrtm_ctx* c, Group& gr, const float* d) {
    CHK(build_tiles(c, gr, c->tile));
    CHK(fill(c, c->pool + c->bg_region, gr.sc_used));
    CHK(fill(c, c->pool + c->bg_region + c->sc_region, gr.img_used));
    const int nt = c->g.nt;
    const bool fz = c->fused;
    // parity of the adjoint fields: number of reverse steps done
    auto apar = [&](int n) { return fz ? (nt - 1 - n) : 0; };
    auto inject = [&](int n) -> lsrtm_status {
        tbeg(c, 7);
        hipError_t e = launch_inject(desc(gr, apar(n)), gr.d_node_slot, gr.d_node_idx, gr.d_node_ptr,
                                     gr.d_node_rec, gr.nnode, n, d, c->st);
        tend(c);
        if (e != hipSuccess) FAIL(c, LSRTM_EHIP, "inject: %s", hipGetErrorString(e));
        return LSRTM_OK;
    };
    tstep(c, nt - 1);
    CHK(inject(nt - 1));
    // segments j >= jc replay into the replay cache, and only when it does
    // not hold this group's replays yet
    const int jc = c->nseg - c->rc_m;
    for (int j = c->nseg - 1; j >= 0; --j) {
        const int n0 = j * c->k, n1 = std::min(n0 + c->k, nt);
        const Slot* rcd = j >= jc ? gr.d_rc + (long long)(j - jc) * gr.ns : nullptr;
        tstep(c, n0);
        if (!rcd || !gr.rc_valid) {
            if (j == 0) CHK(fill(c, c->pool, gr.bg_used));
            else CHK(ckpt(c, gr, j, false, desc(gr, fz ? n0 : 0)));
            for (int n = n0; n < n1; ++n) {
                tstep(c, n);
                const Slot* cur = rcd ? rcd : desc(gr, fz ? n : 0);
                CHK(stencil(c, gr, K_SEG_V, n, n - n0, 0, cur));
                if (!fz) CHK(stencil(c, gr, K_SEG_P, n, n - n0, 0, cur));
            }
        }
        // 2D: the adjoint velocity kernel of step n injects the data of step
        // n - 1 into the new adjoint pressure; 3D uses the injection kernel
        const TileRec tr{gr.d_trp, gr.d_trec, nullptr, d};
        const TileRec none{nullptr, nullptr, nullptr, nullptr};
        for (int n = n1 - 1; n >= n0; --n) {
            tstep(c, n);
            if (n < nt - 1 && c->ndim == 3) CHK(inject(n));
            const Slot* cur = rcd ? rcd : desc(gr, apar(n));
            CHK(stencil(c, gr, K_ADJ_A, n, n - n0, n == nt - 1 ? 1 : 0, cur, fz ? tr : none));
            if (!fz) CHK(stencil(c, gr, K_ADJ_B, n, n - n0, 0, cur, tr));
        }
    }
    ImgArgs ia;
    ia.slots = gr.d_slots;
    ia.win = gr.d_win;
    ia.nslot = gr.ns;
    ia.ndim = c->ndim;
    for (int a = 0; a < 3; ++a) ia.gn[a] = c->g.n[a];
    ia.npml = c->g.npml;
    ia.acc = c->acc64;
    ia.gpts = c->gpts;
    HIPCHK(c, launch_image_reduce(ia, c->st));
    return LSRTM_OK;
}

// Pseudo-Hessian pass of one group (appendix B): the background of every
// shot with the squared velocity increments and squared divergences summed
// over time into the slots' w_a and g_kappa arrays, then added per physical
// node into acc64 in shot order.  Always the two-phase kernels (the fused
// 2D step has no accumulating variant); plain launches.
lsrtm_status group_ph(lsrtm_ctx* c, Group& gr) {
    CHK(build_tiles(c, gr, c->tile));
    CHK(fill(c, c->pool, gr.bg_used));
    CHK(fill(c, c->pool + c->bg_region, gr.sc_used));
    CHK(fill(c, c->pool + c->bg_region + c->sc_region, gr.img_used));
    const Slot* sl = desc(gr, 0);
    for (int n = 0; n < c->g.nt; ++n) {
        tstep(c, n);
        CHK(stencil(c, gr, K_BG_V, n, 0, PH_ACCUMULATE, sl));
        CHK(stencil(c, gr, K_BG_P, n, 0, PH_ACCUMULATE, sl));
    }
    ImgArgs ia;
    ia.slots = gr.d_slots;
    ia.win = gr.d_win;
    ia.nslot = gr.ns;
    ia.ndim = c->ndim;
    for (int a = 0; a < 3; ++a) ia.gn[a] = c->g.n[a];
    ia.npml = c->g.npml;
    ia.acc = c->acc64;
    ia.gpts = c->gpts;
    HIPCHK(c, launch_ph_reduce(ia, c->st));
    return LSRTM_OK;
}

// Passes are captured into one HIP graph per (pass, launch group, data
// pointer, checkpoint flag) and replayed on later calls; with per-launch
// timing requested they run as plain launches.  Graph replay is used when
// the group's launches are short enough for launch overhead to matter.
enum { P_FWD = 0, P_BORN = 1, P_FWDCK = 2, P_ADJ = 3 };

lsrtm_status run_direct(lsrtm_ctx* c, Group& gr, int pass, float* d, bool write_ck) {
    if (pass == P_ADJ) return group_adjoint(c, gr, d);
    return group_forward(c, gr, pass == P_BORN ? 1 : (pass == P_FWDCK ? 2 : 0), d, write_ck);
}

bool use_graph(const lsrtm_ctx* c) {
    return c->opt_graph && !c->opt_timing && (long long)c->groups.size() * c->g.nt <= 400000;
}

lsrtm_status run_group_impl(lsrtm_ctx* c, Group& gr, int gi, int pass, float* d, bool write_ck) {
    if (!use_graph(c)) return run_direct(c, gr, pass, d, write_ck);
    CHK(build_tiles(c, gr, c->tile));
    if (!c->gst) {
        HIPCHK(c, hipStreamCreateWithFlags(&c->gst, hipStreamNonBlocking));
        HIPCHK(c, hipEventCreateWithFlags(&c->gin, hipEventDisableTiming));
        HIPCHK(c, hipEventCreateWithFlags(&c->gout, hipEventDisableTiming));
    }
    // a migration pass that fills the replay cache and one that reads it are
    // different graphs, and so are Born passes with and without it
    const int rcv = (pass == P_ADJ || pass == P_BORN) && gr.rc_valid ? 1 : 0;
    const auto key = std::make_tuple((pass * 2 + (write_ck ? 1 : 0)) * 2 + rcv, gi, (const void*)d, c->tile);
    auto it = c->graphs.find(key);
    hipGraphExec_t exec = nullptr;
    if (it == c->graphs.end()) {
        // a caller that hands in a new data buffer on every call (a training
        // loop through the autograd operator) would otherwise add a graph per
        // call: keep the most recently used ones, four per launch group and
        // pass kind in use (a replaced graph is destroyed after the stream
        // has finished its last launch)
        const size_t cap = c->graph_cap ? c->graph_cap : 8 * c->groups.size() + 8;
        if (c->graphs.size() >= cap) {
            HIPCHK(c, hipStreamSynchronize(c->gst));
            while (c->graphs.size() >= cap && !c->graph_lru.empty()) {
                auto old = c->graphs.find(c->graph_lru.front());
                if (old != c->graphs.end()) {
                    (void)hipGraphExecDestroy(old->second);
                    c->graphs.erase(old);
                }
                c->graph_lru.pop_front();
            }
        }
        hipStream_t user = c->st;
        HIPCHK(c, hipStreamBeginCapture(c->gst, hipStreamCaptureModeThreadLocal));
        c->st = c->gst;
        lsrtm_status s = run_direct(c, gr, pass, d, write_ck);
        c->st = user;
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(c->gst, &graph);
        if (s != LSRTM_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return s;
        }
        if (e != hipSuccess) FAIL(c, LSRTM_EHIP, "graph capture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) FAIL(c, LSRTM_EHIP, "graph instantiate: %s", hipGetErrorString(e));
        c->graphs[key] = exec;
        c->graph_lru.push_back(key);
    } else {
        exec = it->second;
        c->graph_lru.remove(key);
        c->graph_lru.push_back(key);
    }
    HIPCHK(c, hipEventRecord(c->gin, c->st));
    HIPCHK(c, hipStreamWaitEvent(c->gst, c->gin, 0));
    HIPCHK(c, hipGraphLaunch(exec, c->gst));
    HIPCHK(c, hipEventRecord(c->gout, c->gst));
    HIPCHK(c, hipStreamWaitEvent(c->st, c->gout, 0));
    return LSRTM_OK;
}

// One pass of one launch group; with the progress option the pass is waited
// for and reported on stderr.
lsrtm_status run_group(lsrtm_ctx* c, Group& gr, int gi, int pass, float* d, bool write_ck) {
    CHK(run_group_impl(c, gr, gi, pass, d, write_ck));
    // the pass just queued leaves the group's replays in the cache (stream order)
    if (pass == P_ADJ && c->rc_m > 0) gr.rc_valid = true;
    if (c->opt_progress) {
        static const char* name[4] = {"forward", "Born", "background", "migration"};
        HIPCHK(c, hipStreamSynchronize(c->st));
        fprintf(stderr, "[lsrtm] %s pass: group %d of %zu done\n", name[pass], gi + 1, c->groups.size());
        fflush(stderr);
    }
    return LSRTM_OK;
}

lsrtm_status ensure_ckpts(lsrtm_ctx* c) {
    if (c->ckpt_valid) return LSRTM_OK;
    for (auto& gr : c->groups) CHK(group_forward(c, gr, 2, nullptr, true));
    CHK(check_flag(c));
    c->ckpt_valid = true;
    return LSRTM_OK;
}

lsrtm_status autotune(lsrtm_ctx* c, int nsteps, bool groups, double* out);
lsrtm_status plan(lsrtm_ctx* c);

lsrtm_status check_ready(lsrtm_ctx* c) {
    if (!c) return LSRTM_EINVAL;
    if (!c->have_model) FAIL(c, LSRTM_ESTATE, "set_model has not been called");
    if (!c->have_acq) FAIL(c, LSRTM_ESTATE, "set_acquisition has not been called");
    if (c->opt_tile >= 0) {
        c->tile = c->opt_tile;
    } else if (!c->tuned) {
        c->tile = default_tile(c->ndim);
        CHK(autotune(c, 4, false, nullptr));
    }
    return LSRTM_OK;
}

lsrtm_status prep_model_windows(lsrtm_ctx* c) {
    // host tables stay alive until the stream synchronisation below
    std::vector<std::vector<float>> tabs;
    tabs.reserve(3 * c->wins.size());
    for (auto& w : c->wins) {
        PrepArgs a;
        a.lnvp = c->lnvp;
        a.lnip = c->lnip;
        for (int i = 0; i < 3; ++i) {
            a.gn[i] = c->g.n[i];
            a.lo[i] = w.lo[i];
            a.wn[i] = w.hi[i] - w.lo[i];
            a.N[i] = w.N[i];
        }
        a.npml = c->g.npml;
        a.sx = w.sx;
        a.sy = w.sy;
        a.dt = c->g.dt;
        a.ndim = c->ndim;
        a.kdt = w.kdt;
        a.sb = w.sb;
        for (int i = 0; i < 3; ++i) a.bdt[i] = w.bdt[i];
        HIPCHK(c, launch_model_prep(a, c->st));
        // CPML tables
        for (int ax = 0; ax < c->ndim; ++ax) {
            std::vector<float> ach, bch, aci, bci;
            cpml_axis(w.N[ax], c->g.npml, c->g.h[ax], c->g.dt, c->vmax, c->g.pml_R, c->g.pml_f0, true, ach, bch);
            cpml_axis(w.N[ax], c->g.npml, c->g.h[ax], c->g.dt, c->vmax, c->g.pml_R, c->g.pml_f0, false, aci, bci);
            tabs.emplace_back();
            std::vector<float>& tab = tabs.back();
            tab.insert(tab.end(), ach.begin(), ach.end());
            tab.insert(tab.end(), bch.begin(), bch.end());
            tab.insert(tab.end(), aci.begin(), aci.end());
            tab.insert(tab.end(), bci.begin(), bci.end());
            HIPCHK(c, hipMemcpyAsync(w.cpml[ax], tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice, c->st));
        }
    }
    HIPCHK(c, hipStreamSynchronize(c->st));
    background_changed(c);
    return LSRTM_OK;
}

lsrtm_status plan(lsrtm_ctx* c) {
    const int nshot = c->nshot;
    const int* win = c->a_win.data();
    const int* src = c->a_src.data();
    const int* rec_ptr = c->a_recptr.data();
    const int* rec = c->a_rec.data();
    const float* wavelet = c->wavelet;
    HIPCHK(c, hipStreamSynchronize(c->st));
    free_acq(c);
    const int nd = c->ndim;
    const int npml = c->g.npml;
    c->nshot = nshot;
    c->shots.resize(nshot);
    c->h_win.assign(6 * nshot, 0);
    std::map<std::vector<int>, int> wid;
    c->data_len = 0;
    c->padded_total = 0;
    for (int s = 0; s < nshot; ++s) {
        int lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
        for (int a = 0; a < nd; ++a) {
            lo[a] = win[s * 2 * nd + 2 * a];
            hi[a] = win[s * 2 * nd + 2 * a + 1];
            if (lo[a] < 0 || hi[a] > c->g.n[a] || hi[a] <= lo[a])
                FAIL(c, LSRTM_EINVAL, "shot %d: window [%d,%d) on axis %d outside the grid", s, lo[a], hi[a], a);
        }
        std::vector<int> key(lo, lo + 3);
        key.insert(key.end(), hi, hi + 3);
        int w;
        auto it = wid.find(key);
        if (it == wid.end()) {
            Window W;
            for (int a = 0; a < 3; ++a) {
                W.lo[a] = lo[a];
                W.hi[a] = hi[a];
                W.N[a] = a < nd ? hi[a] - lo[a] + 2 * npml : 1;
            }
            W.ldz = (int)round_up(W.N[0], 32);
            W.sx = W.ldz;
            W.sy = W.sx * W.N[1];
            W.npts = W.sy * W.N[2];
            // the stencil kernels address a shot's arrays with 32-bit byte offsets
            if (W.npts >= (1LL << 30))
                FAIL(c, LSRTM_EINVAL, "shot %d: padded window of %lld nodes; at most 2^30 - 1 per shot", s,
                     W.npts);
            // a 3D tile carries its first and last plane in 16 bits each
            if (W.N[2] > 0xffff)
                FAIL(c, LSRTM_EINVAL, "shot %d: padded window of %d planes along y; at most 65535", s, W.N[2]);
            w = (int)c->wins.size();
            wid[key] = w;
            c->wins.push_back(W);
        } else {
            w = it->second;
        }
        const Window& W = c->wins[w];
        for (int a = 0; a < 3; ++a) {
            c->h_win[6 * s + 2 * a] = lo[a];
            c->h_win[6 * s + 2 * a + 1] = hi[a];
        }
        ShotInfo& sh = c->shots[s];
        sh.win = w;
        auto lin = [&](const int* p, long long* out) -> bool {
            long long i = 0;
            const long long strides[3] = {1, W.sx, W.sy};
            for (int a = 0; a < nd; ++a) {
                if (p[a] < lo[a] || p[a] >= hi[a]) return false;
                i += strides[a] * (p[a] - lo[a] + npml);
            }
            *out = i;
            return true;
        };
        long long si;
        if (!lin(src + s * nd, &si)) FAIL(c, LSRTM_EINVAL, "shot %d: source outside its window", s);
        sh.src_lin = (int)si;
        sh.rec0 = rec_ptr[s];
        sh.nrec = rec_ptr[s + 1] - rec_ptr[s];
        sh.rec_lin.resize(sh.nrec);
        for (int r = 0; r < sh.nrec; ++r) {
            long long ri;
            if (!lin(rec + (long long)(sh.rec0 + r) * nd, &ri))
                FAIL(c, LSRTM_EINVAL, "shot %d: receiver %d outside its window", s, r);
            sh.rec_lin[r] = (int)ri;
        }
        sh.data_off = (long long)c->g.nt * sh.rec0;
        c->data_len += (long long)c->g.nt * sh.nrec;
        c->padded_total += (long long)W.N[0] * W.N[1] * W.N[2];
        long long ck = (long long)(1 + nd) * W.npts * (c->g.ckpt_dtype == 0 ? 4 : 2);
        for (int a = 0; a < nd; ++a) ck += 2 * strip_count_h(W.N, a, c->S) * 4;
        sh.ckbytes = round_up(ck, 256);
    }

    // ---- memory plan --------------------------------------------------------
    size_t fr = 0, tot = 0;
    HIPCHK(c, hipMemGetInfo(&fr, &tot));
    const long long budget = c->opt_budget_mb > 0 ? c->opt_budget_mb * 1024LL * 1024LL : (long long)(0.9 * fr);
    c->fused = nd == 2 && c->opt_fused;
    const int nbg = 1 + 3 * nd + (c->fused ? 1 + 2 * nd : 0);   // p, v, psi, phi [, p', v', psi']
    const int nsc = 1 + 3 * nd + (c->fused ? 1 + 3 * nd : 0);   // q, w, xi, eta [, q', w', xi', eta']
    const int nt = c->g.nt;
    long long model_bytes = 0;
    for (auto& W : c->wins) model_bytes += (long long)(4 + (c->fused ? nd : 0)) * W.npts * 4 + 4LL * nd * 4 * std::max(W.N[0], std::max(W.N[1], W.N[2]));
    long long ck_per_shot_sum = 0;
    for (auto& sh : c->shots) ck_per_shot_sum += sh.ckbytes;
    const long long fixed = model_bytes + 2LL * c->gpts * 8 + (long long)nshot * nt * 4 + 2 * c->data_len * 4 +
                            2 * 2 * c->gpts * 4 + (64LL << 20) + (long long)nshot * (1 + nd) * 64 * 4;
    long long max_ck = 0, max_npts = 0;
    for (auto& sh : c->shots) max_ck = std::max(max_ck, sh.ckbytes);
    for (auto& W : c->wins) max_npts = std::max(max_npts, W.npts);
    // Two checkpoint layouts: every shot keeps its checkpoints for the whole
    // lifetime of the plan (written once, reused by every pass), or, when that
    // does not fit, only the shots of the active launch group hold them and
    // each migration pass first re-runs the group's background.
    const int G0 = c->opt_spl > 0 ? std::min(c->opt_spl, nshot) : nshot;
    int G = G0, k = 1;
    long long need = 0;
    bool ckg = false, fits = false;
    for (int mode = c->opt_ckg ? 1 : 0; mode < 2 && !fits; ++mode) {
        ckg = mode == 1;
        G = G0;
        for (;;) {
            long long grp_pts = 0;
            {
                int s = 0;
                for (int gs : group_sizes(nshot, G)) {
                    long long cur = 0;
                    for (int e = 0; e < gs; ++e, ++s) cur += c->wins[c->shots[s].win].npts;
                    grp_pts = std::max(grp_pts, cur);
                }
            }
            const long long seg_step = grp_pts * (nd + 1) * 4;
            const double ck_mem = ckg ? (double)G * max_ck : (double)ck_per_shot_sum;
            if (c->g.ckpt_every > 0) {
                k = std::min(c->g.ckpt_every, nt);
            } else {
                const double kk = std::sqrt((double)nt * ck_mem / (double)std::max(1LL, seg_step));
                k = (int)std::max(1.0, std::min((double)nt, std::round(kk)));
            }
            const int nseg = (nt + k - 1) / k;
            need = fixed + grp_pts * (nbg + nsc + 2) * 4LL + (long long)k * seg_step +
                   (long long)((nseg - 1) * ck_mem) + (long long)nseg * nshot * (1 + nd) * 4;
            if (need <= budget) {
                fits = true;
                break;
            }
            if (G == 1) break;
            G = (G + 1) / 2;
        }
    }
    if (!fits)
        FAIL(c, LSRTM_ENOMEM, "memory plan needs %.2f GB, budget %.2f GB", need / 1e9, budget / 1e9);
    // With a replay cache (whole segments only), a checkpoint interval the
    // planner chose may shrink, down to half, when the cache then holds more
    // steps; results do not depend on the interval.
    if (c->opt_rcache_mb > 0 && !c->fused && !ckg && c->g.ckpt_every <= 0) {
        long long grp_pts = 0, all_pts = 0;
        {
            int s = 0;
            for (int gs : group_sizes(nshot, G)) {
                long long cur = 0;
                for (int e = 0; e < gs; ++e, ++s) cur += c->wins[c->shots[s].win].npts;
                grp_pts = std::max(grp_pts, cur);
                all_pts += cur;
            }
        }
        const long long seg_step = grp_pts * (nd + 1) * 4;   // replay buffer bytes per step
        const long long step_all = all_pts * (nd + 1) * 4;   // cache bytes per step, all groups
        auto need_of = [&](int kk) -> long long {
            const int ns = (nt + kk - 1) / kk;
            return fixed + grp_pts * (nbg + nsc + 2) * 4LL + (long long)kk * seg_step +
                   (long long)((ns - 1) * (double)ck_per_shot_sum) + (long long)ns * nshot * (1 + nd) * 4;
        };
        auto held = [&](int kk) -> long long {   // steps of every group the cache would hold
            const long long nk = need_of(kk);
            if (nk > budget) return -1;
            const long long cap = std::min(c->opt_rcache_mb * 1024LL * 1024LL, budget - nk);
            const int ns = (nt + kk - 1) / kk;
            const long long m = std::min<long long>(ns, cap / ((long long)kk * step_all));
            return m >= ns ? nt : m * kk;
        };
        int bk = k;
        long long best = held(k);
        for (int kk = k - 1; kk >= std::max(1, k / 2); --kk) {
            const long long h = held(kk);
            if (h > best) {
                best = h;
                bk = kk;
            }
        }
        if (bk != k) {
            k = bk;
            need = need_of(k);
        }
    }
    c->ck_group = ckg;
    c->G = group_sizes(nshot, G)[0];
    c->k = k;
    c->nseg = (nt + k - 1) / k;
    c->plan_bytes = need;

    // ---- model windows -------------------------------------------------------
    for (auto& W : c->wins) {
        CHK(dalloc_t(c, &W.kdt, W.npts, true));
        CHK(dalloc_t(c, &W.sb, W.npts, true));
        // the stored dt b_a products serve only the fused 2D adjoint
        for (int a = 0; a < 3; ++a) {
            if (a < nd && c->fused) CHK(dalloc_t(c, &W.bdt[a], W.npts, true));
            else W.bdt[a] = nullptr;
            if (a < nd) CHK(dalloc_t(c, &W.cpml[a], 4 * W.N[a], true));
            else W.cpml[a] = nullptr;
        }
        CHK(dalloc_t(c, &W.dlnr, W.npts, true));
        CHK(dalloc_t(c, &W.dlnk, W.npts, true));
        HIPCHK(c, launch_fill(W.kdt, W.npts, 0.f, c->st));
        HIPCHK(c, launch_fill(W.dlnr, W.npts, 0.f, c->st));
        HIPCHK(c, launch_fill(W.dlnk, W.npts, 0.f, c->st));
        HIPCHK(c, launch_fill(W.sb, W.npts, 0.f, c->st));
        for (int a = 0; a < nd; ++a)
            if (W.bdt[a]) HIPCHK(c, launch_fill(W.bdt[a], W.npts, 0.f, c->st));
    }
    // ---- groups ----------------------------------------------------------------
    int s0 = 0;
    for (int gs : group_sizes(nshot, G)) {
        Group gr;
        gr.s0 = s0;
        gr.ns = gs;
        s0 += gs;
        long long pts = 0;
        for (int s = gr.s0; s < gr.s0 + gr.ns; ++s) pts += c->wins[c->shots[s].win].npts;
        gr.bg_used = pts * nbg;
        gr.sc_used = pts * nsc;
        gr.img_used = pts * 2;
        c->bg_region = std::max(c->bg_region, gr.bg_used);
        c->sc_region = std::max(c->sc_region, gr.sc_used);
        c->img_region = std::max(c->img_region, gr.img_used);
        c->groups.push_back(gr);
    }
    long long seg_floats = 0;
    for (auto& gr : c->groups) {
        long long pts = gr.bg_used / nbg;
        seg_floats = std::max(seg_floats, (long long)c->k * (nd + 1) * pts);
    }
    CHK(dalloc_t(c, &c->pool, c->bg_region + c->sc_region + c->img_region, true));
    CHK(dalloc_t(c, &c->segbuf, seg_floats, true));
    // Replay cache: the replays of the last rc_m segments of every group are
    // kept across passes in HBM the budget leaves over (they depend on the
    // background only, like the checkpoints) and read by later migration and
    // 2D Born passes.  Two-phase steps with checkpoints held for the whole
    // plan only.
    long long rc_seg = 0;          // floats of one cached segment over all groups
    for (auto& gr : c->groups) rc_seg += (long long)c->k * (nd + 1) * (gr.bg_used / nbg);
    if (c->opt_rcache_mb > 0 && !c->fused && !c->ck_group && rc_seg > 0) {
        const long long cap = std::min(c->opt_rcache_mb * 1024LL * 1024LL, budget - need);
        c->rc_m = (int)std::max(0LL, std::min((long long)c->nseg, cap / (rc_seg * 4)));
        if (c->rc_m > 0) CHK(dalloc_t(c, &c->rcache, (size_t)c->rc_m * rc_seg, true));
        c->plan_bytes += (long long)c->rc_m * rc_seg * 4;
    }
    const long long ck_total = c->ck_group ? (long long)(c->nseg - 1) * G * max_ck : (long long)(c->nseg - 1) * ck_per_shot_sum;
    CHK(dalloc(c, reinterpret_cast<void**>(&c->ckbuf), (size_t)std::max(1LL, ck_total), true));
    CHK(dalloc_t(c, &c->ckscales, (size_t)c->nseg * nshot * (1 + nd), true));
    // blocks per field of a snapshot's max-abs pass: enough for the pass to
    // fill the GPU (about 8192 blocks) also when a group holds one or a few
    // large shots; the maximum is exact in any order, so this changes no scale
    c->nblk = (int)std::min<long long>(1024, std::max<long long>(64, (8192 + (1 + nd) * G - 1) / ((1 + nd) * G)));
    CHK(dalloc_t(c, &c->ckpart, (size_t)G * (1 + nd) * c->nblk, true));
    CHK(dalloc_t(c, &c->acc64, 2 * c->gpts, true));
    CHK(dalloc_t(c, &c->src_amp, (size_t)nshot * nt, true));
    CHK(dalloc_t(c, &c->cg_r, std::max(1LL, c->data_len), true));
    CHK(dalloc_t(c, &c->cg_w, std::max(1LL, c->data_len), true));
    CHK(dalloc_t(c, &c->cg_z, 2 * c->gpts, true));
    CHK(dalloc_t(c, &c->cg_p, 2 * c->gpts, true));
    HIPCHK(c, launch_fill(c->pool, c->bg_region + c->sc_region + c->img_region, 0.f, c->st));
    HIPCHK(c, launch_fill(c->src_amp, (long long)nshot * nt, 0.f, c->st));
    double cell = 1.0;
    for (int a = 0; a < nd; ++a) cell *= c->g.h[a];
    HIPCHK(c, launch_axpy(c->g.dt / cell, wavelet, c->src_amp, (long long)nshot * nt, c->st));

    // checkpoint offsets per shot: [j][shot] blocks -> shot-major inside each j
    // is not needed; each shot owns nseg consecutive checkpoints.
    std::vector<long long> ckoff(nshot);
    {
        long long o = 0;
        for (int s = 0; s < nshot; ++s) {
            ckoff[s] = o;
            o += (long long)(c->nseg - 1) * c->shots[s].ckbytes;
        }
    }
    // descriptors, receivers
    long long rc_base = 0;         // floats of the replay cache taken by earlier groups
    for (auto& gr : c->groups) {
        long long obg = 0, osc = 0, oimg = 0, oseg = 0;
        float* bgb = c->pool;
        float* scb = c->pool + c->bg_region;
        float* imb = c->pool + c->bg_region + c->sc_region;
        std::vector<Rec> recs;
        std::vector<int> wins6;
        std::vector<std::pair<long long, int>> nodes;   // (slot<<32 | idx, rec index)
        for (int i = 0; i < gr.ns; ++i) {
            const int s = gr.s0 + i;
            const ShotInfo& sh = c->shots[s];
            const Window& W = c->wins[sh.win];
            Slot S;
            memset(&S, 0, sizeof(S));
            for (int a = 0; a < 3; ++a) S.n[a] = W.N[a];
            S.ldz = W.ldz;
            S.sx = W.sx;
            S.sy = W.sy;
            S.npts = W.npts;
            S.src = sh.src_lin;
            S.shot = s;
            S.npml = c->g.npml;
            S.src_amp = c->src_amp + (long long)s * nt;
            S.kdt = W.kdt;
            S.sb = W.sb;
            for (int a = 0; a < 3; ++a) {
                S.bdt[a] = W.bdt[a];
                S.cpml[a] = W.cpml[a];
            }
            S.dlnr = W.dlnr;
            S.dlnk = W.dlnk;
            float* b = bgb + obg;
            S.p = b;
            for (int a = 0; a < 3; ++a) {
                const bool on = a < nd;
                S.v[a] = on ? b + (1 + a) * W.npts : nullptr;
                S.psi[a] = on ? b + (1 + nd + a) * W.npts : nullptr;
                S.phi[a] = on ? b + (1 + 2 * nd + a) * W.npts : nullptr;
            }
            float* q = scb + osc;
            S.q = q;
            for (int a = 0; a < 3; ++a) {
                const bool on = a < nd;
                S.w[a] = on ? q + (1 + a) * W.npts : nullptr;
                S.xi[a] = on ? q + (1 + nd + a) * W.npts : nullptr;
                S.eta[a] = on ? q + (1 + 2 * nd + a) * W.npts : nullptr;
            }
            if (c->fused) {
                S.pn = b + (1 + 3 * nd) * W.npts;
                S.qn = q + (1 + 3 * nd) * W.npts;
                for (int a = 0; a < nd; ++a) {
                    S.vn[a] = b + (2 + 3 * nd + a) * W.npts;
                    S.psin[a] = b + (2 + 4 * nd + a) * W.npts;
                    S.wn[a] = q + (2 + 3 * nd + a) * W.npts;
                    S.xin[a] = q + (2 + 4 * nd + a) * W.npts;
                    S.etan[a] = q + (2 + 5 * nd + a) * W.npts;
                }
            }
            S.gk = imb + oimg;
            S.gr = imb + oimg + W.npts;
            S.seg = c->segbuf + oseg;
            if (c->ck_group) {
                S.ck = c->ckbuf + (long long)i * (c->nseg - 1) * max_ck;
                S.ckbytes = max_ck;
            } else {
                S.ck = c->ckbuf + ckoff[s];
                S.ckbytes = sh.ckbytes;
            }
            obg += (long long)nbg * W.npts;
            osc += (long long)nsc * W.npts;
            oimg += 2LL * W.npts;
            oseg += (long long)c->k * (nd + 1) * W.npts;
            gr.max_npts = std::max(gr.max_npts, W.npts);
            gr.h_slots.push_back(S);
            for (int r = 0; r < sh.nrec; ++r) {
                Rec R;
                R.slot = i;
                R.idx = sh.rec_lin[r];
                R.out = sh.data_off + r;
                R.stride = sh.nrec;
                R.pad = 0;
                nodes.push_back({((long long)i << 32) | (unsigned)R.idx, (int)recs.size()});
                recs.push_back(R);
            }
            for (int a = 0; a < 6; ++a) wins6.push_back(c->h_win[6 * s + a]);
        }
        CHK(dalloc_t(c, &gr.d_slots, gr.ns, true));
        HIPCHK(c, hipMemcpy(gr.d_slots, gr.h_slots.data(), gr.ns * sizeof(Slot), hipMemcpyHostToDevice));
        if (c->rc_m > 0) {
            // cached segment m of this group: its slots' replay buffers at the
            // offsets they have in segbuf, inside block m of the group's range
            const long long gseg = (long long)c->k * (nd + 1) * (gr.bg_used / nbg);
            std::vector<Slot> rc;
            for (int m = 0; m < c->rc_m; ++m)
                for (const Slot& S0 : gr.h_slots) {
                    Slot S = S0;
                    S.seg = c->rcache + rc_base + m * gseg + (S0.seg - c->segbuf);
                    rc.push_back(S);
                }
            CHK(dalloc_t(c, &gr.d_rc, rc.size(), true));
            HIPCHK(c, hipMemcpy(gr.d_rc, rc.data(), rc.size() * sizeof(Slot), hipMemcpyHostToDevice));
            rc_base += (long long)c->rc_m * gseg;
        }
        if (c->fused) {
            std::vector<Slot> alt = gr.h_slots;
            for (Slot& S : alt) {
                std::swap(S.p, S.pn);
                std::swap(S.q, S.qn);
                for (int a = 0; a < 3; ++a) {
                    std::swap(S.v[a], S.vn[a]);
                    std::swap(S.psi[a], S.psin[a]);
                    std::swap(S.w[a], S.wn[a]);
                    std::swap(S.xi[a], S.xin[a]);
                    std::swap(S.eta[a], S.etan[a]);
                }
            }
            CHK(dalloc_t(c, &gr.d_alt, gr.ns, true));
            HIPCHK(c, hipMemcpy(gr.d_alt, alt.data(), gr.ns * sizeof(Slot), hipMemcpyHostToDevice));
        }
        CHK(dalloc_t(c, &gr.d_win, wins6.size(), true));
        HIPCHK(c, hipMemcpy(gr.d_win, wins6.data(), wins6.size() * sizeof(int), hipMemcpyHostToDevice));
        gr.nrec = (int)recs.size();
        gr.h_rec = recs;
        CHK(dalloc_t(c, &gr.d_rec, std::max<size_t>(1, recs.size()), true));
        if (!recs.empty())
            HIPCHK(c, hipMemcpy(gr.d_rec, recs.data(), recs.size() * sizeof(Rec), hipMemcpyHostToDevice));
        // distinct receiver nodes (stable order: receivers of one node keep
        // their shot order)
        std::stable_sort(nodes.begin(), nodes.end(),
                         [](const std::pair<long long, int>& a, const std::pair<long long, int>& b) {
                             return a.first < b.first;
                         });
        std::vector<int> nslot, nidx, nptr;
        std::vector<Rec> nrec;
        for (size_t i = 0; i < nodes.size(); ++i) {
            if (i == 0 || nodes[i].first != nodes[i - 1].first) {
                nslot.push_back((int)(nodes[i].first >> 32));
                nidx.push_back((int)(nodes[i].first & 0xffffffffLL));
                nptr.push_back((int)nrec.size());
            }
            nrec.push_back(recs[nodes[i].second]);
        }
        nptr.push_back((int)nrec.size());
        gr.nnode = (int)nslot.size();
        CHK(dalloc_t(c, &gr.d_node_slot, std::max<size_t>(1, nslot.size()), true));
        CHK(dalloc_t(c, &gr.d_node_idx, std::max<size_t>(1, nidx.size()), true));
        CHK(dalloc_t(c, &gr.d_node_ptr, nptr.size(), true));
        CHK(dalloc_t(c, &gr.d_node_rec, std::max<size_t>(1, nrec.size()), true));
        if (!nslot.empty()) {
            HIPCHK(c, hipMemcpy(gr.d_node_slot, nslot.data(), nslot.size() * sizeof(int), hipMemcpyHostToDevice));
            HIPCHK(c, hipMemcpy(gr.d_node_idx, nidx.data(), nidx.size() * sizeof(int), hipMemcpyHostToDevice));
            HIPCHK(c, hipMemcpy(gr.d_node_rec, nrec.data(), nrec.size() * sizeof(Rec), hipMemcpyHostToDevice));
        }
        HIPCHK(c, hipMemcpy(gr.d_node_ptr, nptr.data(), nptr.size() * sizeof(int), hipMemcpyHostToDevice));
    }
    c->have_acq = true;
    CHK(prep_model_windows(c));
    return LSRTM_OK;
}



// ---------------------------------------------------------------------------
// Autotuner: times the six stencil phases over a few steps on the real launch
// groups for every tile shape (and, when asked, several group sizes) and
// keeps the fastest.  Results are cached per problem shape in the file named
// by LSRTM_TUNE_CACHE when that variable is set.
// ---------------------------------------------------------------------------
std::string tune_key(const lsrtm_ctx* c) {
    char b[256];
    snprintf(b, sizeof(b), "nd=%d nshot=%d pts=%lld nt=%d n=%dx%dx%d npml=%d", c->ndim, c->nshot,
             c->padded_total, c->g.nt, c->g.n[0], c->g.n[1], c->g.n[2], c->g.npml);
    return b;
}

bool tune_cache_get(const lsrtm_ctx* c, int* tile, int* spl, int* fused, int* tile_v, int* tile_a) {
    const char* f = getenv("LSRTM_TUNE_CACHE");
    if (!f) return false;
    FILE* fp = fopen(f, "r");
    if (!fp) return false;
    const std::string key = tune_key(c);
    char line[512];
    bool found = false;
    while (fgets(line, sizeof(line), fp)) {
        std::string l(line);
        const size_t bar = l.find('|');
        if (bar == std::string::npos || l.substr(0, bar) != key) continue;
        int t, g, f, tv = -1, ta = -1;
        if (sscanf(l.c_str() + bar + 1, "%d %d %d %d %d", &t, &g, &f, &tv, &ta) >= 3) {
            *tile = t;
            *spl = g;
            *fused = f;
            *tile_v = tv;
            *tile_a = ta;
            found = true;
        }
    }
    fclose(fp);
    return found;
}

void tune_cache_put(const lsrtm_ctx* c, int tile, int spl, int fused) {
    const char* f = getenv("LSRTM_TUNE_CACHE");
    if (!f) return;
    FILE* fp = fopen(f, "a");
    if (!fp) return;
    fprintf(fp, "%s|%d %d %d %d %d\n", tune_key(c).c_str(), tile, spl, fused, c->opt_tile_v, c->opt_tile_a);
    fclose(fp);
}

// Milliseconds per time step of the six stencil phases summed over all groups.
lsrtm_status time_tile(lsrtm_ctx* c, int tile, int nsteps, double* ms) {
    c->tile = tile;
    hipEvent_t a, b;
    HIPCHK(c, hipEventCreate(&a));
    HIPCHK(c, hipEventCreate(&b));
    for (auto& gr : c->groups) CHK(build_tiles(c, gr, tile));
    const bool tim = c->opt_timing;
    c->opt_timing = 0;
    HIPCHK(c, hipEventRecord(a, c->st));
    // the passes' order per group: Born steps, then replayed background
    // steps, then adjoint steps, so that what stays cached between launches
    // is what stays cached in a real pass
    for (auto& gr : c->groups) {
        for (int n = 0; n < nsteps; ++n) {
            const Slot* sl = desc(gr, c->fused ? n : 0);
            CHK(stencil(c, gr, K_BORN_V, n, 0, 0, sl));
            if (!c->fused) CHK(stencil(c, gr, K_BORN_P, n, 0, 0, sl));
        }
        for (int n = 0; n < nsteps; ++n) {
            const Slot* sl = desc(gr, c->fused ? n : 0);
            CHK(stencil(c, gr, K_SEG_V, n, n % c->k, 0, sl));
            if (!c->fused) CHK(stencil(c, gr, K_SEG_P, n, n % c->k, 0, sl));
        }
        for (int n = 0; n < nsteps; ++n) {
            const Slot* sl = desc(gr, c->fused ? n : 0);
            CHK(stencil(c, gr, K_ADJ_A, n, n % c->k, n == 0, sl));
            if (!c->fused) CHK(stencil(c, gr, K_ADJ_B, n, n % c->k, 0, sl));
        }
    }
    HIPCHK(c, hipEventRecord(b, c->st));
    HIPCHK(c, hipEventSynchronize(b));
    float t = 0.f;
    HIPCHK(c, hipEventElapsedTime(&t, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    c->opt_timing = tim;
    *ms = t / nsteps;
    return LSRTM_OK;
}

lsrtm_status tune_tiles(lsrtm_ctx* c, int nsteps, int* best, double* best_ms) {
    const int ntile = c->ndim == 2 ? kNumTiles2 : kNumTiles3;
    // zero the working fields so that the timing runs on finite values
    for (auto& gr : c->groups) {
        CHK(fill(c, c->pool, gr.bg_used));
        CHK(fill(c, c->pool + c->bg_region, gr.sc_used));
        CHK(fill(c, c->pool + c->bg_region + c->sc_region, gr.img_used));
    }
    double ms;
    // one shape for every phase first
    c->opt_tile_v = c->opt_tile_a = -1;
    CHK(time_tile(c, 0, 1, &ms));   // warm-up
    *best = 0;
    *best_ms = 1e30;
    for (int t = 0; t < ntile; ++t) {
        CHK(time_tile(c, t, nsteps, &ms));
        if (ms < *best_ms) {
            *best_ms = ms;
            *best = t;
        }
    }
    c->tile = *best;
    // then, for two-phase steps, the phases without receivers may keep
    // shapes of their own: the velocity phases, then the adjoint A phase
    if (!c->fused) {
        for (int* opt : {&c->opt_tile_v, &c->opt_tile_a}) {
            int pick = -1;
            for (int t = 0; t < ntile; ++t) {
                if (t == *best) continue;
                *opt = t;
                CHK(time_tile(c, *best, nsteps, &ms));
                if (ms < *best_ms) {
                    *best_ms = ms;
                    pick = t;
                }
            }
            *opt = pick;
        }
    }
    clear_graphs(c);
    return LSRTM_OK;
}

lsrtm_status autotune(lsrtm_ctx* c, int nsteps, bool groups, double* out) {
    int tile = -1, spl = c->opt_spl, fused = c->opt_fused, tile_v = -1, tile_a = -1;
    if (tune_cache_get(c, &tile, &spl, &fused, &tile_v, &tile_a)) {
        if (groups && (spl != c->opt_spl || fused != c->opt_fused)) {
            c->opt_spl = spl;
            c->opt_fused = fused;
            CHK(plan(c));
        }
        c->tile = tile;
        c->opt_tile_v = tile_v;
        c->opt_tile_a = tile_a;
        c->tuned = true;
        clear_graphs(c);
        if (out) {
            out[0] = tile;
            out[1] = c->G;
            out[2] = -1.0;
            out[3] = tile_v;
            out[4] = tile_a;
        }
        return LSRTM_OK;
    }
    double best_ms = 1e30;
    int best_tile = 0, best_spl = c->opt_spl, best_fused = c->opt_fused, best_tv = -1, best_ta = -1;
    std::vector<int> cands;
    if (groups) {
        cands.push_back(0);
        for (int g : {64, 48, 32, 24, 16, 8})
            if (g < c->nshot) cands.push_back(g);
    } else {
        cands.push_back(c->opt_spl);
    }
    // 2D: both schedules (fused one-kernel steps and two-phase steps)
    std::vector<int> scheds;
    if (groups && c->ndim == 2) scheds = {1, 0};
    else scheds = {c->opt_fused};
    for (int f : scheds) {
        for (int g : cands) {
            if (g != c->opt_spl || f != c->opt_fused) {
                c->opt_spl = g;
                c->opt_fused = f;
                CHK(plan(c));
            }
            int t;
            double ms;
            CHK(tune_tiles(c, nsteps, &t, &ms));
            if (ms < best_ms) {
                best_ms = ms;
                best_tile = t;
                best_spl = g;
                best_fused = f;
                best_tv = c->opt_tile_v;
                best_ta = c->opt_tile_a;
            }
        }
    }
    if (best_spl != c->opt_spl || best_fused != c->opt_fused) {
        c->opt_spl = best_spl;
        c->opt_fused = best_fused;
        CHK(plan(c));
    }
    c->tile = best_tile;
    c->opt_tile_v = best_tv;
    c->opt_tile_a = best_ta;
    c->tuned = true;
    clear_graphs(c);
    tune_cache_put(c, best_tile, best_spl, best_fused);
    if (out) {
        out[0] = best_tile;
        out[1] = c->G;
        out[2] = best_ms;
        out[3] = best_tv;
        out[4] = best_ta;
    }
    return LSRTM_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* lsrtm_strerror(int s) {
    switch (s) {
    case LSRTM_OK: return "ok";
    case LSRTM_EINVAL: return "invalid argument";
    case LSRTM_ENOMEM: return "out of device memory";
    case LSRTM_EHIP: return "HIP runtime error";
    case LSRTM_EUNSTABLE: return "CFL stability condition violated";
    case LSRTM_ENONFINITE: return "non-finite value";
    case LSRTM_ESTATE: return "call out of order";
    default: return "unknown status";
    }
}

const char* lsrtm_last_error(lsrtm_ctx* c) { return c ? c->err.c_str() : ""; }

lsrtm_status lsrtm_tile_shape(int ndim, int id, int* out) {
    if (!out) return LSRTM_EINVAL;
    if (ndim == 2 && id >= 0 && id < kNumTiles2) {
        out[0] = kTiles2[id][0];
        out[1] = kTiles2[id][1];
        return LSRTM_OK;
    }
    if (ndim == 3 && id >= 0 && id < kNumTiles3) {
        out[0] = kTiles3[id][0];
        out[1] = kTiles3[id][1];
        return LSRTM_OK;
    }
    return LSRTM_EINVAL;
}

lsrtm_status lsrtm_create(const lsrtm_grid* g, void* stream, lsrtm_ctx** out) {
    if (!g || !out) return LSRTM_EINVAL;
    *out = nullptr;
    if (g->ndim != 2 && g->ndim != 3) return LSRTM_EINVAL;
    for (int a = 0; a < g->ndim; ++a)
        if (g->n[a] < 1 || !(g->h[a] > 0.0)) return LSRTM_EINVAL;
    if (g->ndim == 2 && g->n[2] != 1) return LSRTM_EINVAL;
    if (g->npml < 0 || g->nt < 1 || !(g->dt > 0.0)) return LSRTM_EINVAL;
    if (g->npml > 0 && !(g->pml_R > 0.0 && g->pml_R < 1.0)) return LSRTM_EINVAL;
    if (g->ckpt_every < 0 || g->ckpt_dtype < 0 || g->ckpt_dtype > 2) return LSRTM_EINVAL;
    lsrtm_ctx* c = new lsrtm_ctx();
    c->g = *g;
    if (g->ndim == 2) c->g.h[2] = 1.0;
    c->st = reinterpret_cast<hipStream_t>(stream);
    c->ndim = g->ndim;
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 4; ++k) c->C.c[a][k] = (float)(kC8[k] / c->g.h[a]);
    c->gpts = (long long)g->n[0] * g->n[1] * g->n[2];
    c->S = strip_depth(c);
    *out = c;
    return LSRTM_OK;
}

void lsrtm_destroy(lsrtm_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->st);
    free_acq(c);
    if (c->wavelet) (void)hipFree(c->wavelet);
    if (c->gst) (void)hipStreamDestroy(c->gst);
    if (c->gin) (void)hipEventDestroy(c->gin);
    if (c->gout) (void)hipEventDestroy(c->gout);
    for (void* p : c->allocs) (void)hipFree(p);
    for (auto& e : c->evpool) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    if (c->pa) (void)hipEventDestroy(c->pa);
    if (c->pb) (void)hipEventDestroy(c->pb);
    wiener_free(c->wiener);
    delete c;
}

// sizes in MB beyond any device (2^30 MB = 1 PiB), so that MB * 2^20 never overflows
constexpr long long kMaxMB = 1LL << 30;

lsrtm_status lsrtm_set_option(lsrtm_ctx* c, int key, long long v) {
    if (!c) return LSRTM_EINVAL;
    switch (key) {
    case LSRTM_OPT_SHOTS_PER_LAUNCH:
        if (v < 0 || v > INT_MAX) FAIL(c, LSRTM_EINVAL, "shots per launch must be in [0, %d]", INT_MAX);
        if (c->opt_spl == (int)v) return LSRTM_OK;
        c->opt_spl = (int)v;
        if (c->have_acq) return plan(c);   // rebuild the launch groups
        return LSRTM_OK;
    case LSRTM_OPT_TILE: {
        const int nt = c->ndim == 2 ? kNumTiles2 : kNumTiles3;
        if (v < -1 || v >= nt) FAIL(c, LSRTM_EINVAL, "tile id %lld out of range", v);
        c->opt_tile = (int)v;
        c->tile = (int)v;
        c->tuned = v >= 0;
        clear_graphs(c);
        return LSRTM_OK;
    }
    case LSRTM_OPT_GRAPH: c->opt_graph = v != 0; return LSRTM_OK;
    case LSRTM_OPT_TIMING: c->opt_timing = v != 0; return LSRTM_OK;
    case LSRTM_OPT_MEM_BUDGET_MB:
        if (v < 0 || v > kMaxMB) FAIL(c, LSRTM_EINVAL, "memory budget must be in [0, %lld] MB", kMaxMB);
        c->opt_budget_mb = v;
        return LSRTM_OK;
    case LSRTM_OPT_FUSED:
        if (c->opt_fused == (v != 0)) return LSRTM_OK;
        c->opt_fused = v != 0;
        if (c->have_acq) return plan(c);
        return LSRTM_OK;
    case LSRTM_OPT_PROGRESS: c->opt_progress = v != 0; return LSRTM_OK;
    case LSRTM_OPT_TILE_V:
    case LSRTM_OPT_TILE_ADJ_A: {
        const int nt = c->ndim == 2 ? kNumTiles2 : kNumTiles3;
        if (v < -1 || v >= nt) FAIL(c, LSRTM_EINVAL, "tile id %lld out of range", v);
        (key == LSRTM_OPT_TILE_V ? c->opt_tile_v : c->opt_tile_a) = (int)v;
        clear_graphs(c);
        return LSRTM_OK;
    }
    case LSRTM_OPT_GRAPH_CACHE:
        if (v < 0 || v > INT_MAX) FAIL(c, LSRTM_EINVAL, "graph cache size must be in [0, %d]", INT_MAX);
        c->graph_cap = (size_t)v;
        return LSRTM_OK;
    case LSRTM_OPT_REPLAY_CACHE_MB:
        if (v < 0 || v > kMaxMB) FAIL(c, LSRTM_EINVAL, "replay cache size must be in [0, %lld] MB", kMaxMB);
        if (c->opt_rcache_mb == v) return LSRTM_OK;
        c->opt_rcache_mb = v;
        if (c->have_acq) return plan(c);
        return LSRTM_OK;
    case LSRTM_OPT_CKPT_PER_GROUP:
        if (c->opt_ckg == (v != 0)) return LSRTM_OK;
        c->opt_ckg = v != 0;
        if (c->have_acq) return plan(c);
        return LSRTM_OK;
    default: FAIL(c, LSRTM_EINVAL, "unknown option %d", key);
    }
}

lsrtm_status lsrtm_set_model(lsrtm_ctx* c, const float* lnvp, const float* lnip) {
    if (!c || !lnvp || !lnip) return LSRTM_EINVAL;
    if (!c->lnvp) {
        CHK(dalloc_t(c, &c->lnvp, c->gpts, false));
        CHK(dalloc_t(c, &c->lnip, c->gpts, false));
        CHK(dalloc_t(c, &c->partial, 8 * 256 * 4, false));
        CHK(dalloc_t(c, &c->dpart, 1024, false));
        CHK(dalloc_t(c, &c->dscal, 16, false));
        CHK(dalloc_t(c, &c->d_flag, 64, false));
        HIPCHK(c, launch_fill(reinterpret_cast<float*>(c->d_flag), 64, 0.f, c->st));
    }
    HIPCHK(c, hipMemcpyAsync(c->lnvp, lnvp, c->gpts * sizeof(float), hipMemcpyDeviceToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->lnip, lnip, c->gpts * sizeof(float), hipMemcpyDeviceToDevice, c->st));
    // vmax and finiteness
    const int nb = 256;
    std::vector<float> part(nb);
    HIPCHK(c, launch_maxval(c->lnvp, c->gpts, c->partial, nb, c->st));
    HIPCHK(c, hipMemcpyAsync(part.data(), c->partial, nb * sizeof(float), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    float mv = -INFINITY;
    for (float x : part) mv = std::max(mv, x);
    HIPCHK(c, launch_maxval(c->lnip, c->gpts, c->partial, nb, c->st));
    HIPCHK(c, hipMemcpyAsync(part.data(), c->partial, nb * sizeof(float), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    float mi = -INFINITY;
    for (float x : part) mi = std::max(mi, x);
    if (!std::isfinite(mv) || !std::isfinite(mi)) {
        c->have_model = false;
        FAIL(c, LSRTM_ENONFINITE, "model holds NaN or Inf");
    }
    // the same reduction with negated sign is not needed: logs are finite
    const double vmax = std::exp((double)mv);
    double s2 = 0.0;
    for (int a = 0; a < c->ndim; ++a) s2 += 1.0 / (c->g.h[a] * c->g.h[a]);
    double csum = 0.0;
    for (double x : kC8) csum += std::fabs(x);
    const double cfl = vmax * c->g.dt * std::sqrt(s2) * csum;
    if (!(cfl < 1.0)) {
        c->have_model = false;
        FAIL(c, LSRTM_EUNSTABLE, "CFL number %.4f >= 1 (vmax %.1f m/s, dt %g s)", cfl, vmax, c->g.dt);
    }
    c->vmax = vmax;
    c->have_model = true;
    if (c->have_acq) CHK(prep_model_windows(c));
    background_changed(c);
    return LSRTM_OK;
}

lsrtm_status lsrtm_set_acquisition(lsrtm_ctx* c, int nshot, const int* win, const int* src,
                                   const int* rec_ptr, const int* rec, const float* wavelet) {
    if (!c) return LSRTM_EINVAL;
    if (!c->have_model) FAIL(c, LSRTM_ESTATE, "set_model must precede set_acquisition");
    if (nshot < 1 || !win || !src || !rec_ptr || !wavelet) FAIL(c, LSRTM_EINVAL, "bad acquisition arguments");
    if (rec_ptr[0] != 0) FAIL(c, LSRTM_EINVAL, "rec_ptr[0] must be 0");
    for (int s = 0; s < nshot; ++s)
        if (rec_ptr[s + 1] < rec_ptr[s]) FAIL(c, LSRTM_EINVAL, "rec_ptr must be non-decreasing");
    if (rec_ptr[nshot] > 0 && !rec) FAIL(c, LSRTM_EINVAL, "rec is NULL");
    const int nd = c->ndim;
    HIPCHK(c, hipStreamSynchronize(c->st));
    c->a_win.assign(win, win + (size_t)nshot * 2 * nd);
    c->a_src.assign(src, src + (size_t)nshot * nd);
    c->a_recptr.assign(rec_ptr, rec_ptr + nshot + 1);
    c->a_rec.assign(rec ? rec : rec_ptr, rec ? rec + (size_t)rec_ptr[nshot] * nd : rec_ptr);
    if (c->wavelet) {
        (void)hipFree(c->wavelet);
        c->wavelet = nullptr;
    }
    c->nshot = nshot;
    {
        hipError_t e = hipMalloc(&c->wavelet, (size_t)nshot * c->g.nt * sizeof(float));
        if (e != hipSuccess) FAIL(c, LSRTM_ENOMEM, "wavelet copy: %s", hipGetErrorString(e));
    }
    HIPCHK(c, hipMemcpyAsync(c->wavelet, wavelet, (size_t)nshot * c->g.nt * sizeof(float),
                             hipMemcpyDeviceToDevice, c->st));
    c->tuned = false;
    return plan(c);
}

lsrtm_status lsrtm_autotune(lsrtm_ctx* c, int nsteps, int tune_groups, double* out) {
    if (!c) return LSRTM_EINVAL;
    if (!c->have_model || !c->have_acq) FAIL(c, LSRTM_ESTATE, "autotune needs a model and an acquisition");
    if (nsteps < 1) FAIL(c, LSRTM_EINVAL, "nsteps must be >= 1");
    c->opt_tile = -1;
    CHK(autotune(c, nsteps, tune_groups != 0, out));
    background_changed(c);
    return LSRTM_OK;
}

lsrtm_status lsrtm_sizes(lsrtm_ctx* c, long long* out, int nout) {
    if (!c || !out) return LSRTM_EINVAL;
    long long v[14] = {c->data_len, c->gpts, c->G, c->k, (long long)c->groups.size(), c->padded_total, c->plan_bytes,
                       c->tile, c->ck_group ? 1 : 0, c->fused ? 1 : 0, c->opt_tile_v, c->opt_tile_a, c->rc_m,
                       (long long)c->graphs.size()};
    for (int i = 0; i < nout && i < 14; ++i) out[i] = v[i];
    return LSRTM_OK;
}

lsrtm_status lsrtm_stats(lsrtm_ctx* c, double* out, int nout) {
    if (!c || !out) return LSRTM_EINVAL;
    std::vector<double> v(1 + 2 * LSRTM_NKERNEL);
    v[0] = c->pass_ms;
    for (int i = 0; i < LSRTM_NKERNEL; ++i) {
        v[1 + 2 * i] = c->kms[i];
        v[2 + 2 * i] = (double)c->kcnt[i];
    }
    for (int i = 0; i < nout && i < (int)v.size(); ++i) out[i] = v[i];
    return LSRTM_OK;
}

lsrtm_status lsrtm_forward(lsrtm_ctx* c, float* d) {
    CHK(check_ready(c));
    if (!d && c->data_len > 0) FAIL(c, LSRTM_EINVAL, "d is NULL");
    CHK(pass_begin(c));
    for (size_t gi = 0; gi < c->groups.size(); ++gi)
        CHK(run_group(c, c->groups[gi], (int)gi, P_FWD, d, !c->ck_group));
    CHK(pass_end(c));
    CHK(check_flag(c));
    c->ckpt_valid = !c->ck_group;
    return LSRTM_OK;
}

static lsrtm_status born_impl(lsrtm_ctx* c, const float* dm, float* d) {
    for (auto& W : c->wins) {
        DmArgs a;
        a.dm = dm;
        a.gpts = c->gpts;
        for (int i = 0; i < 3; ++i) {
            a.gn[i] = c->g.n[i];
            a.lo[i] = W.lo[i];
            a.wn[i] = W.hi[i] - W.lo[i];
            a.N[i] = W.N[i];
        }
        a.npml = c->g.npml;
        a.sx = W.sx;
        a.sy = W.sy;
        a.ndim = c->ndim;
        a.dlnr = W.dlnr;
        a.dlnk = W.dlnk;
        HIPCHK(c, launch_dm_prep(a, c->st));
    }
    const bool write_ck = !c->ckpt_valid && !c->ck_group;
    for (size_t gi = 0; gi < c->groups.size(); ++gi) CHK(run_group(c, c->groups[gi], (int)gi, P_BORN, d, write_ck));
    if (write_ck) {
        CHK(check_flag(c));
        c->ckpt_valid = true;
    }
    return LSRTM_OK;
}

lsrtm_status lsrtm_born(lsrtm_ctx* c, const float* dm, float* d) {
    CHK(check_ready(c));
    if (!dm || (!d && c->data_len > 0)) FAIL(c, LSRTM_EINVAL, "NULL argument");
    CHK(pass_begin(c));
    CHK(born_impl(c, dm, d));
    CHK(pass_end(c));
    return LSRTM_OK;
}

static lsrtm_status adjoint_impl(lsrtm_ctx* c, const float* d, float* img, int accumulate) {
    if (!c->ck_group) CHK(ensure_ckpts(c));
    HIPCHK(c, launch_fill_f64(c->acc64, 2 * c->gpts, c->st));
    for (size_t gi = 0; gi < c->groups.size(); ++gi) {
        if (c->ck_group) CHK(run_group(c, c->groups[gi], (int)gi, P_FWDCK, nullptr, true));
        CHK(run_group(c, c->groups[gi], (int)gi, P_ADJ, const_cast<float*>(d), false));
    }
    if (c->ck_group) CHK(check_flag(c));
    HIPCHK(c, launch_image_store(c->acc64, img, 2 * c->gpts, accumulate, c->st));
    return LSRTM_OK;
}

lsrtm_status lsrtm_adjoint(lsrtm_ctx* c, const float* d, float* img, int accumulate) {
    CHK(check_ready(c));
    if (!img || (!d && c->data_len > 0)) FAIL(c, LSRTM_EINVAL, "NULL argument");
    CHK(pass_begin(c));
    CHK(adjoint_impl(c, d, img, accumulate));
    CHK(pass_end(c));
    return LSRTM_OK;
}

static lsrtm_status dot_impl(lsrtm_ctx* c, const float* a, const float* b, long long n, double* out) {
    double r = 0.0;
    if (n > 0) {
        HIPCHK(c, launch_dot(a, b, n, c->dpart, 1024, c->dscal, c->st));
        HIPCHK(c, hipMemcpyAsync(&r, c->dscal, sizeof(double), hipMemcpyDeviceToHost, c->st));
        HIPCHK(c, hipStreamSynchronize(c->st));
    }
    *out = r;
    return LSRTM_OK;
}

lsrtm_status lsrtm_dot(lsrtm_ctx* c, const float* a, const float* b, long long n, double* out) {
    if (!c || !out || n < 0 || (n > 0 && (!a || !b))) return LSRTM_EINVAL;
    if (!c->dpart) {
        CHK(dalloc_t(c, &c->dpart, 1024, false));
        CHK(dalloc_t(c, &c->dscal, 16, false));
    }
    return dot_impl(c, a, b, n, out);
}

lsrtm_status lsrtm_axpy(lsrtm_ctx* c, double alpha, const float* x, float* y, long long n) {
    if (!c || n < 0 || (n > 0 && (!x || !y))) return LSRTM_EINVAL;
    HIPCHK(c, launch_axpy(alpha, x, y, n, c->st));
    return LSRTM_OK;
}

lsrtm_status lsrtm_stream_mix(lsrtm_ctx* c, float* buf, long long n, int nread, int nwrite, const int* grid,
                              double* ms) {
    if (!c || !buf || !ms || n < 1) return LSRTM_EINVAL;
    const int key = nread * 16 + nwrite;
    if (key != 10 * 16 + 6 && key != 10 * 16 + 2 && key != 5 * 16 + 6 && key != 5 * 16 + 2 && key != 2 * 16 + 1)
        FAIL(c, LSRTM_EINVAL, "stream_mix: unsupported mix (%d reads, %d writes)", nread, nwrite);
    if (grid && (grid[0] < 1 || grid[1] < 1 || grid[2] < 1 || grid[0] > grid[3] ||
                 (long long)grid[3] * grid[1] * grid[2] != n))
        FAIL(c, LSRTM_EINVAL, "stream_mix: grid does not match n = ldz * nx * ny with nz <= ldz");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(c, hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    if (e == hipSuccess) e = launch_stream_mix(buf, n, nread, nwrite, grid, c->st, e0, e1);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) FAIL(c, LSRTM_EHIP, "stream_mix: %s", hipGetErrorString(e));
    *ms = t;
    return LSRTM_OK;
}

// z = M^-1 L^T r (preconditioned run: s = L^T r kept), or z = L^T r.
static lsrtm_status normal_residual(lsrtm_ctx* c) {
    const long long nm = 2 * c->gpts;
    if (!c->cg_pre) return adjoint_impl(c, c->cg_r, c->cg_z, 0);
    CHK(adjoint_impl(c, c->cg_r, c->cg_s, 0));
    HIPCHK(c, launch_mul(c->cg_minv, c->cg_s, c->cg_z, nm, c->st));
    return LSRTM_OK;
}

lsrtm_status lsrtm_cgnr_begin(lsrtm_ctx* c, const float* d_obs, float* x) {
    CHK(check_ready(c));
    if (!x || (!d_obs && c->data_len > 0)) FAIL(c, LSRTM_EINVAL, "bad CGNR arguments");
    const long long nm = 2 * c->gpts, nd = c->data_len;
    CHK(pass_begin(c));
    c->cg_pre = c->precond;
    HIPCHK(c, launch_copy(d_obs, c->cg_r, nd, c->st));
    HIPCHK(c, launch_fill(x, nm, 0.f, c->st));
    CHK(normal_residual(c));
    HIPCHK(c, launch_copy(c->cg_z, c->cg_p, nm, c->st));
    CHK(dot_impl(c, c->cg_z, c->cg_pre ? c->cg_s : c->cg_z, nm, &c->cg_zz));
    CHK(dot_impl(c, c->cg_r, c->cg_r, nd, &c->cg_r0));
    c->cg_rr = c->cg_r0;
    c->cg_k = 0;
    c->cg_alpha = c->cg_beta = c->cg_ww = 0.0;
    c->cg_active = true;
    CHK(pass_end(c));
    return LSRTM_OK;
}

lsrtm_status lsrtm_cgnr_iterate(lsrtm_ctx* c, float* x, double* misfit) {
    CHK(check_ready(c));
    if (!c->cg_active) FAIL(c, LSRTM_ESTATE, "lsrtm_cgnr_begin has not been called");
    if (!x) FAIL(c, LSRTM_EINVAL, "x is NULL");
    const long long nm = 2 * c->gpts, nd = c->data_len;
    CHK(pass_begin(c));
    c->cg_alpha = c->cg_beta = c->cg_ww = 0.0;
    if (c->cg_zz > 0.0 && c->cg_r0 > 0.0) {
        CHK(born_impl(c, c->cg_p, c->cg_w));
        double ww;
        CHK(dot_impl(c, c->cg_w, c->cg_w, nd, &ww));
        c->cg_ww = ww;
        if (ww > 0.0) {
            const double alpha = c->cg_zz / ww;
            c->cg_alpha = alpha;
            HIPCHK(c, launch_axpy(alpha, c->cg_p, x, nm, c->st));
            HIPCHK(c, launch_axpy(-alpha, c->cg_w, c->cg_r, nd, c->st));
            CHK(normal_residual(c));
            double zz1;
            CHK(dot_impl(c, c->cg_z, c->cg_pre ? c->cg_s : c->cg_z, nm, &zz1));
            const double beta = zz1 / c->cg_zz;
            c->cg_beta = beta;
            HIPCHK(c, launch_xpby(c->cg_z, beta, c->cg_p, nm, c->st));
            c->cg_zz = zz1;
        }
        CHK(dot_impl(c, c->cg_r, c->cg_r, nd, &c->cg_rr));
    }
    c->cg_k += 1;
    if (misfit) *misfit = c->cg_r0 > 0.0 ? c->cg_rr / c->cg_r0 : 0.0;
    CHK(pass_end(c));
    return LSRTM_OK;
}

lsrtm_status lsrtm_cgnr(lsrtm_ctx* c, const float* d_obs, int niter, float* x, double* misfit) {
    if (!c) return LSRTM_EINVAL;
    if (niter < 0) FAIL(c, LSRTM_EINVAL, "niter < 0");
    CHK(lsrtm_cgnr_begin(c, d_obs, x));
    if (misfit) misfit[0] = 1.0;
    for (int it = 0; it < niter; ++it) CHK(lsrtm_cgnr_iterate(c, x, misfit ? misfit + it + 1 : nullptr));
    return LSRTM_OK;
}

lsrtm_status lsrtm_cgnr_step(lsrtm_ctx* c, double* out) {
    if (!c || !out) return LSRTM_EINVAL;
    if (!c->cg_active) FAIL(c, LSRTM_ESTATE, "no CGNR run");
    out[0] = (double)c->cg_k;
    out[1] = c->cg_alpha;
    out[2] = c->cg_beta;
    out[3] = c->cg_ww;
    out[4] = c->cg_r0 > 0.0 ? c->cg_rr / c->cg_r0 : 0.0;
    return LSRTM_OK;
}

lsrtm_status lsrtm_cgnr_state(lsrtm_ctx* c, int get, float* r, float* z, float* p, double* scal) {
    CHK(check_ready(c));
    if (!r || !z || !p || !scal) FAIL(c, LSRTM_EINVAL, "NULL argument");
    const long long nm = 2 * c->gpts, nd = c->data_len;
    if (get) {
        if (!c->cg_active) FAIL(c, LSRTM_ESTATE, "no CGNR run to export");
        HIPCHK(c, launch_copy(c->cg_r, r, nd, c->st));
        HIPCHK(c, launch_copy(c->cg_z, z, nm, c->st));
        HIPCHK(c, launch_copy(c->cg_p, p, nm, c->st));
        scal[0] = c->cg_zz;
        scal[1] = c->cg_r0;
        scal[2] = c->cg_rr;
        scal[3] = (double)c->cg_k;
        HIPCHK(c, hipStreamSynchronize(c->st));
    } else {
        HIPCHK(c, launch_copy(r, c->cg_r, nd, c->st));
        HIPCHK(c, launch_copy(z, c->cg_z, nm, c->st));
        HIPCHK(c, launch_copy(p, c->cg_p, nm, c->st));
        c->cg_zz = scal[0];
        c->cg_r0 = scal[1];
        c->cg_rr = scal[2];
        c->cg_k = (int)scal[3];
        c->cg_alpha = c->cg_beta = c->cg_ww = 0.0;
        c->cg_active = true;
        c->cg_pre = c->precond;
    }
    return LSRTM_OK;
}

// Corner/weight tables of the interpolated PSF Hessian for a lattice spacing
// (appendix C): scatterers at W, W + s, ... on every axis, W = (s - 1) / 2;
// coordinate j lies between corners c0 <= c1 with weight (j - c0) / s,
// clamped to [0, 1] outside the lattice.
static lsrtm_status psf_setup(lsrtm_ctx* c, const float* psf, int spacing, int mono, PsfArgs* a) {
    if (spacing < 1) FAIL(c, LSRTM_EINVAL, "PSF spacing must be >= 1");
    const int W = (spacing - 1) / 2;
    a->ndim = c->ndim;
    a->W = W;
    a->mono = mono ? 1 : 0;
    a->N = c->gpts;
    a->psf = psf;
    long long tot = 0;
    for (int ax = 0; ax < 3; ++ax) {
        a->n[ax] = ax < c->ndim ? c->g.n[ax] : 1;
        a->off[ax] = (int)tot;
        tot += a->n[ax];
    }
    if (!c->psf_tab) CHK(dalloc_t(c, &c->psf_tab, 3 * (size_t)tot, false));
    a->tab = c->psf_tab;
    if (c->psf_spacing == spacing) return LSRTM_OK;
    std::vector<int> tab(3 * tot, 0);
    for (int ax = 0; ax < c->ndim; ++ax) {
        const int n = a->n[ax];
        std::vector<int> lat;
        for (int v = W; v < n; v += spacing) lat.push_back(v);
        if (lat.empty()) FAIL(c, LSRTM_EINVAL, "PSF spacing %d leaves no scatterer on axis %d (%d nodes)", spacing, ax, n);
        for (int j = 0; j < n; ++j) {
            int c0, c1;
            double w;
            if (lat.size() == 1) {
                c0 = c1 = lat[0];
                w = 0.0;
            } else {
                long long k = (long long)std::floor((double)(j - lat[0]) / spacing);
                k = std::min<long long>(std::max<long long>(k, 0), (long long)lat.size() - 2);
                c0 = lat[k];
                c1 = lat[k + 1];
                w = std::min(1.0, std::max(0.0, (double)(j - c0) / spacing));
            }
            const float wf = (float)w;
            int* t = &tab[3 * (a->off[ax] + j)];
            t[0] = c0;
            t[1] = c1;
            memcpy(&t[2], &wf, sizeof(float));
        }
    }
    HIPCHK(c, hipMemcpy(c->psf_tab, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice));
    c->psf_spacing = spacing;
    return LSRTM_OK;
}

lsrtm_status lsrtm_psf_images(lsrtm_ctx* c, int spacing, float* psf) {
    CHK(check_ready(c));
    if (!psf) FAIL(c, LSRTM_EINVAL, "psf is NULL");
    PsfArgs a;
    CHK(psf_setup(c, psf, spacing, 0, &a));
    const long long nm = 2 * c->gpts;
    if (!c->psf_dm) CHK(dalloc_t(c, &c->psf_dm, nm, false));
    if (!c->psf_d) CHK(dalloc_t(c, &c->psf_d, std::max(1LL, c->data_len), true));
    CHK(pass_begin(c));
    for (int q = 0; q < 2; ++q) {
        HIPCHK(c, launch_psf_spikes(a, q, c->psf_dm, c->st));
        CHK(born_impl(c, c->psf_dm, c->psf_d));
        CHK(adjoint_impl(c, c->psf_d, psf + (long long)q * nm, 0));
    }
    CHK(pass_end(c));
    return LSRTM_OK;
}

lsrtm_status lsrtm_psf_apply(lsrtm_ctx* c, const float* psf, int spacing, int mono, int transpose,
                             const float* x, float* y) {
    if (!c || !psf || !x || !y) return LSRTM_EINVAL;
    if (x == y) FAIL(c, LSRTM_EINVAL, "x and y must not alias");
    PsfArgs a;
    CHK(psf_setup(c, psf, spacing, mono, &a));
    HIPCHK(c, launch_psf_apply(a, x, y, transpose, c->st));
    return LSRTM_OK;
}

lsrtm_status lsrtm_psf_cgnr(lsrtm_ctx* c, const float* psf, int spacing, int mono, const float* m_rtm, int niter,
                            float* x, double* misfit) {
    if (!c || !psf || !m_rtm || !x) return LSRTM_EINVAL;
    if (niter < 0) FAIL(c, LSRTM_EINVAL, "niter < 0");
    if (!c->dpart) FAIL(c, LSRTM_ESTATE, "set_model must precede lsrtm_psf_cgnr");
    PsfArgs a;
    CHK(psf_setup(c, psf, spacing, mono, &a));
    const long long M = (mono ? 1 : 2) * c->gpts;
    for (int k = 0; k < 4; ++k)
        if (!c->psf_v[k]) CHK(dalloc_t(c, &c->psf_v[k], 2 * c->gpts, false));
    float *r = c->psf_v[0], *z = c->psf_v[1], *p = c->psf_v[2], *w = c->psf_v[3];
    // CGNR on H^T H x = H^T m_rtm (section 3, eq. migdeconobj), x0 = 0
    HIPCHK(c, launch_copy(m_rtm, r, M, c->st));
    HIPCHK(c, launch_fill(x, M, 0.f, c->st));
    HIPCHK(c, launch_psf_apply(a, r, z, 1, c->st));
    HIPCHK(c, launch_copy(z, p, M, c->st));
    double zz, r0;
    CHK(dot_impl(c, z, z, M, &zz));
    CHK(dot_impl(c, r, r, M, &r0));
    double rr = r0;
    if (misfit) misfit[0] = 1.0;
    for (int it = 0; it < niter; ++it) {
        if (zz > 0.0 && r0 > 0.0) {
            HIPCHK(c, launch_psf_apply(a, p, w, 0, c->st));
            double ww;
            CHK(dot_impl(c, w, w, M, &ww));
            if (ww > 0.0) {
                const double alpha = zz / ww;
                HIPCHK(c, launch_axpy(alpha, p, x, M, c->st));
                HIPCHK(c, launch_axpy(-alpha, w, r, M, c->st));
                HIPCHK(c, launch_psf_apply(a, r, z, 1, c->st));
                double zz1;
                CHK(dot_impl(c, z, z, M, &zz1));
                const double beta = zz1 / zz;
                HIPCHK(c, launch_xpby(z, beta, p, M, c->st));
                zz = zz1;
            }
            CHK(dot_impl(c, r, r, M, &rr));
        }
        if (misfit) misfit[it + 1] = r0 > 0.0 ? rr / r0 : 0.0;
    }
    return LSRTM_OK;
}

lsrtm_status lsrtm_mute(lsrtm_ctx* c, float* d, double v_mute, double t0, int ntaper) {
    if (!c) return LSRTM_EINVAL;
    if (!c->have_acq) FAIL(c, LSRTM_ESTATE, "set_acquisition must precede lsrtm_mute");
    if (!(v_mute > 0.0) || ntaper < 0 || !std::isfinite(t0)) FAIL(c, LSRTM_EINVAL, "bad mute parameters");
    if (!d && c->data_len > 0) FAIL(c, LSRTM_EINVAL, "d is NULL");
    const int nd = c->ndim;
    const int total = c->a_recptr[c->nshot];
    if (total == 0) return LSRTM_OK;
    std::vector<long long> off(total);
    std::vector<int> stride(total);
    std::vector<double> tc(total);
    for (int s = 0; s < c->nshot; ++s) {
        const int r0 = c->a_recptr[s], nr = c->a_recptr[s + 1] - r0;
        for (int r = 0; r < nr; ++r) {
            double d2 = 0.0;
            for (int a = 0; a < nd; ++a) {
                const double x = (c->a_rec[(size_t)(r0 + r) * nd + a] - c->a_src[(size_t)s * nd + a]) * c->g.h[a];
                d2 += x * x;
            }
            off[r0 + r] = (long long)c->g.nt * r0 + r;
            stride[r0 + r] = nr;
            tc[r0 + r] = t0 + std::sqrt(d2) / v_mute;
        }
    }
    long long* d_off = nullptr;
    int* d_stride = nullptr;
    double* d_tc = nullptr;
    HIPCHK(c, hipMalloc(&d_off, total * sizeof(long long)));
    hipError_t e = hipMalloc(&d_stride, total * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&d_tc, total * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(d_off, off.data(), total * sizeof(long long), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_stride, stride.data(), total * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_tc, tc.data(), total * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_mute(d, d_off, d_stride, d_tc, total, c->g.nt, c->g.dt, ntaper, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    (void)hipFree(d_off);
    (void)hipFree(d_stride);
    (void)hipFree(d_tc);
    if (e != hipSuccess) FAIL(c, LSRTM_EHIP, "mute: %s", hipGetErrorString(e));
    return LSRTM_OK;
}

// ---------------------------------------------------------------------------
// The mute without allocations: its per-receiver tables (trace offset, row
// length, cut time) are computed on the device from the acquisition the
// plan already holds, into a file-scope device array (one copy per GPU,
// shared by every call on that GPU) instead of buffers allocated per call.
// ---------------------------------------------------------------------------
namespace {
constexpr long long kMuteMaxRec = 1LL << 18;   // receivers over all shots
constexpr long long kMuteScratchBytes = kMuteMaxRec * (8 + 8 + 4);
constexpr int kMaxDevices = 64;
}  // namespace

// In host code this name is a stand-in, not a device address: host code uses
// the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char mute_scratch[kMuteScratchBytes];

static void* g_mute_scratch[kMaxDevices] = {};
static std::mutex g_mute_scratch_mu;

// Device address of mute_scratch on the current device (looked up on the
// first call on each device, then kept).
static lsrtm_status mute_scratch_address(lsrtm_ctx* c, unsigned char** out) {
    int dev = -1;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) FAIL(c, LSRTM_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_mute_scratch_mu);
    if (!g_mute_scratch[dev]) {
        void* p = nullptr;
        HIPCHK(c, hipGetSymbolAddress(&p, HIP_SYMBOL(mute_scratch)));
        if (!p) FAIL(c, LSRTM_EHIP, "no device address for the mute scratch");
        g_mute_scratch[dev] = p;
    }
    *out = static_cast<unsigned char*>(g_mute_scratch[dev]);
    return LSRTM_OK;
}

lsrtm_status lsrtm_mute_noalloc(lsrtm_ctx* c, float* d, double v_mute, double t0, int ntaper) {
    if (!c) return LSRTM_EINVAL;
    if (!c->have_acq) FAIL(c, LSRTM_ESTATE, "set_acquisition must precede lsrtm_mute_noalloc");
    if (!(v_mute > 0.0) || ntaper < 0 || !std::isfinite(t0)) FAIL(c, LSRTM_EINVAL, "bad mute parameters");
    if (!d && c->data_len > 0) FAIL(c, LSRTM_EINVAL, "d is NULL");
    const long long total = c->a_recptr[c->nshot];
    if (total > kMuteMaxRec)
        FAIL(c, LSRTM_EINVAL, "%lld receivers; lsrtm_mute_noalloc handles at most %lld (use lsrtm_mute)", total,
             kMuteMaxRec);
    if (total == 0) return LSRTM_OK;
    unsigned char* scr = nullptr;
    CHK(mute_scratch_address(c, &scr));
    long long* off = reinterpret_cast<long long*>(scr);
    double* tc = reinterpret_cast<double*>(scr + 8 * kMuteMaxRec);
    int* stride = reinterpret_cast<int*>(scr + 16 * kMuteMaxRec);
    long long base = 0;
    for (auto& gr : c->groups) {
        HIPCHK(c, launch_mute_tables(gr.d_slots, gr.d_rec, gr.nrec, c->ndim, c->g.h, t0, v_mute, off + base,
                                     stride + base, tc + base, c->st));
        base += gr.nrec;
    }
    if (base != total) FAIL(c, LSRTM_EHIP, "receiver count mismatch (%lld of %lld)", base, total);
    HIPCHK(c, launch_mute(d, off, stride, tc, (int)total, c->g.nt, c->g.dt, ntaper, c->st));
    return LSRTM_OK;
}

lsrtm_status lsrtm_wiener(lsrtm_ctx* c, const float* m_ref, const float* m_blur, const float* m_in, int nimg,
                          int block, double eps_rel, float* out) {
    if (!c || !m_ref || !m_blur || !m_in || !out || nimg < 1) return LSRTM_EINVAL;
    int n[3];
    for (int a = 0; a < 3; ++a) n[a] = a < c->ndim ? c->g.n[a] : 1;
    const char* err = wiener_apply(&c->wiener, c->ndim, n, block, eps_rel, m_ref, m_blur, m_in, nimg, out, c->st);
    if (err) FAIL(c, strstr(err, "must") ? LSRTM_EINVAL : LSRTM_EHIP, "wiener: %s", err);
    return LSRTM_OK;
}

lsrtm_status lsrtm_set_preconditioner(lsrtm_ctx* c, const float* minv) {
    if (!c) return LSRTM_EINVAL;
    if (!minv) {
        c->precond = false;
        return LSRTM_OK;
    }
    const long long nm = 2 * c->gpts;
    if (!c->cg_minv) {
        CHK(dalloc_t(c, &c->cg_minv, nm, false));
        CHK(dalloc_t(c, &c->cg_s, nm, false));
    }
    HIPCHK(c, launch_copy(minv, c->cg_minv, nm, c->st));
    c->precond = true;
    return LSRTM_OK;
}

lsrtm_status lsrtm_pseudo_hessian(lsrtm_ctx* c, float* h, float* minv, double eps_rel) {
    CHK(check_ready(c));
    if (!h) FAIL(c, LSRTM_EINVAL, "h is NULL");
    if (!(eps_rel >= 0.0)) FAIL(c, LSRTM_EINVAL, "eps_rel must be >= 0");
    CHK(pass_begin(c));
    HIPCHK(c, launch_fill_f64(c->acc64, 2 * c->gpts, c->st));
    const bool fz = c->fused;
    c->fused = false;              // the accumulating kernels are the two-phase ones
    lsrtm_status s = LSRTM_OK;
    for (size_t gi = 0; gi < c->groups.size() && s == LSRTM_OK; ++gi) {
        s = group_ph(c, c->groups[gi]);
        if (s == LSRTM_OK && c->opt_progress) {
            const hipError_t e = hipStreamSynchronize(c->st);
            if (e != hipSuccess) {
                c->fused = fz;
                FAIL(c, LSRTM_EHIP, "pseudo-Hessian pass: %s", hipGetErrorString(e));
            }
            fprintf(stderr, "[lsrtm] pseudo-Hessian pass: group %zu of %zu done\n", gi + 1, c->groups.size());
            fflush(stderr);
        }
    }
    c->fused = fz;
    CHK(s);
    HIPCHK(c, launch_ph_finish(c->acc64, c->lnvp, c->lnip, c->g.dt, h, c->gpts, c->st));
    if (minv) {
        const int nb = 256;
        std::vector<float> part(nb);
        HIPCHK(c, launch_maxval(h, c->gpts, c->partial, nb, c->st));
        HIPCHK(c, hipMemcpyAsync(part.data(), c->partial, nb * sizeof(float), hipMemcpyDeviceToHost, c->st));
        HIPCHK(c, hipStreamSynchronize(c->st));
        float mx = 0.f;
        for (float x : part) mx = std::max(mx, x);
        if (!std::isfinite(mx)) FAIL(c, LSRTM_ENONFINITE, "pseudo-Hessian holds NaN or Inf");
        const double eps = eps_rel * (double)mx;
        if (!(eps > 0.0)) FAIL(c, LSRTM_EINVAL, "zero pseudo-Hessian or eps_rel: preconditioner undefined");
        HIPCHK(c, launch_ph_minv(h, eps, minv, c->gpts, c->st));
    }
    CHK(pass_end(c));
    return LSRTM_OK;
}

}  // extern "C"
