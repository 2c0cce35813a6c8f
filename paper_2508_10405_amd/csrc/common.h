// Device-side data structures shared by the kernels and the runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

namespace lsrtm {

constexpr int HW = 4;        // half width of the eighth-order staggered stencil
constexpr int NTHREADS = 256;
// Flag bit of the background (non-Born, non-replay) velocity and pressure
// kernels: also accumulate the squared velocity increments into the slot's
// w_a arrays and the squared divergence into g_kappa (pseudo-Hessian pass;
// those arrays are free while only the background runs).
constexpr int PH_ACCUMULATE = 2;

// Stencil weights c_k / h_a for the three axes (z, x, y).
struct Coef {
    float c[3][4];
};

// Global (address space 1) element types.  Kernels read the per-shot
// pointers out of a table in device memory, so the compiler cannot tell
// their address space; typing them as global lets it emit global_load /
// global_store instead of flat accesses (which share the LDS counter and
// force waits on both).
using gfloat = __attribute__((address_space(1))) float;
using gchar = __attribute__((address_space(1))) char;

// One shot being advanced by a launch ("slot").  All pointers are device
// pointers into library-owned buffers; arrays are z-fastest with strides
// sx (x) and sy (y) on the shot's padded grid.  The host fills SlotT<0>
// (plain pointers); kernels read the same bytes as SlotT<1> (global).
template <int AS>
struct AddrSpace {
    using F = __attribute__((address_space(AS))) float;
    using C = __attribute__((address_space(AS))) char;
};
template <>
struct AddrSpace<0> {   // the language's default (generic) pointers
    using F = float;
    using C = char;
};

template <int AS>
struct SlotT {
    using F = typename AddrSpace<AS>::F;
    using C = typename AddrSpace<AS>::C;
    int n[3];                // padded sizes (z, x, y); n[2] = 1 in 2D
    int ldz;                 // z stride (== sx)
    long long sx, sy;        // strides of x and y
    long long npts;          // elements per array
    int src;                 // linear index of the source node, -1 for none
    int shot;                // global shot index
    int npml;                // CPML width in nodes (every side, every axis)
    int pad_;
    const F* src_amp;        // [nt] dt * w / cell
    const F* kdt;            // dt * kappa at nodes
    const F* sb;             // sqrt(dt b) at nodes: dt b_a at the half node i + 1/2
                             // is sb[i] * sb[i + e_a] (sb[i]^2 on an axis' last node)
    const F* bdt[3];         // the same products, stored (fused 2D schedule only; else null)
    const F* dlnr;           // dlnrho at nodes (zero in the PML)
    const F* dlnk;           // dlnkappa at nodes (zero in the PML)
    const F* cpml[3];        // per axis: [ach | bch | aci | bci], n_a each
    F* p;                    // background pressure
    F* v[3];                 // background particle velocities
    F* psi[3];               // background CPML memory of G_a p
    F* phi[3];               // background CPML memory of D_a v_a
    F* q;                    // scattered pressure  | adjoint Q = -dt kappa p~
    F* w[3];                 // scattered velocity  | adjoint U_a = -dt b_a v~_a
    F* xi[3];                // scattered psi       | adjoint of psi (chi)
    F* eta[3];               // scattered phi       | adjoint of phi
    F* gk;                   // image of lnkappa
    F* gr;                   // image of lnrho
    // second buffers of the fused one-kernel-per-step schedule: the step
    // reads the fields above and writes the ones below (roles swap every
    // step).  Null when the two-phase schedule is in use.
    F* pn;
    F* vn[3];
    F* psin[3];
    F* qn;
    F* wn[3];
    F* xin[3];
    F* etan[3];
    F* seg;                  // replay buffer [k][ndim + 1][npts]: G_a p + psi_a, q
    C* ck;                   // checkpoint 1 of this shot; checkpoint j >= 1 at ck + (j-1) * ckbytes
    long long ckbytes;
};
using Slot = SlotT<0>;
using DSlot = SlotT<1>;
static_assert(sizeof(Slot) == sizeof(DSlot), "host and device slot layouts differ");

// Device view of a slot table filled by the host.
__host__ __device__ inline const DSlot* dev_slots(const Slot* s) { return reinterpret_cast<const DSlot*>(s); }

// Launch kernel k on stream st.  With an event pair the runtime stamps the
// kernel's own start and end into e0 / e1 (hipExtLaunchKernel), so the
// elapsed time between them is the kernel's execution alone, without the
// marker packets that a separate hipEventRecord would put around it.
template <typename F, typename... A>
inline void launch_k(F k, dim3 g, dim3 b, hipStream_t st, hipEvent_t e0, hipEvent_t e1, A... args) {
    if (e0) hipExtLaunchKernelGGL(k, g, b, 0, st, e0, e1, 0, args...);
    else k<<<g, b, 0, st>>>(args...);
}

// Element i of a device array whose base is uniform over the workgroup (read
// from the slot table), addressed as that base plus a 32-bit byte offset.
// The empty asm makes the offset opaque, so the compiler keeps it as one
// 32-bit register and emits global loads and stores with a scalar base and
// a vector offset (one offset register serves every array read at the same
// node) instead of a 64-bit address per array.  Needs arrays below 4 GiB.
__device__ __forceinline__ unsigned boff(unsigned i) {
    unsigned o = i << 2;
    asm("" : "+v"(o));
    return o;
}
__device__ __forceinline__ gfloat& elem(gfloat* a, unsigned i) {
    return *reinterpret_cast<gfloat*>(reinterpret_cast<gchar*>(a) + boff(i));
}
__device__ __forceinline__ const gfloat& elem(const gfloat* a, unsigned i) {
    return *reinterpret_cast<const gfloat*>(reinterpret_cast<const gchar*>(a) + boff(i));
}

// Receiver entry of a launch group.
struct Rec {
    int slot;
    int idx;                 // linear index in the slot's arrays
    long long out;           // data offset of (it = 0, this receiver)
    int stride;              // nrec of the shot (data row length)
    int pad;
};

// Receivers handled inside the 2D stencil kernels: per tile, the receivers
// whose node lies in the tile (Rec::idx = tile-local node lz + BZ * lx).
struct TileRec {
    const int* ptr;          // [ntiles + 1] ranges into rec; nullptr = none
    const Rec* rec;
    float* d;                // record the new pressure here (forward / Born)
    const float* y;          // inject y[n - 1] into the new adjoint pressure
};

// Record v for every receiver of tile tix at tile-local node e, step n.
__device__ __forceinline__ void tile_gather(const TileRec& tr, int tix, int e, int n, float v) {
    const int r1 = tr.ptr[tix + 1];
    for (int j = tr.ptr[tix]; j < r1; ++j) {
        const Rec R = tr.rec[j];
        if (R.idx == e) tr.d[R.out + (long long)n * R.stride] = v;
    }
}

// Sum of the data of step n over the receivers of tile tix at node e (in
// list order).
__device__ __forceinline__ float tile_inject(const TileRec& tr, int tix, int e, int n) {
    float s = 0.f;
    const int r1 = tr.ptr[tix + 1];
    for (int j = tr.ptr[tix]; j < r1; ++j) {
        const Rec R = tr.rec[j];
        if (R.idx == e) s = s + tr.y[R.out + (long long)n * R.stride];
    }
    return s;
}

// Blocks are dispatched round-robin over the 8 XCDs (block b on XCD b % 8);
// give every XCD a contiguous range of tiles so that neighbouring tiles,
// which share halos, meet in the same L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
    const int xcd = bid & 7, k = bid >> 3;
    const int per = nblocks >> 3, rem = nblocks & 7;
    const int base = xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per;
    return base + k;
}

// A set of cells (tile-local row lz, column lx; negative = halo) that the
// block stages: rows ZL + jz (jz < NZ) and columns XL + jx (jx < NX), where
// an index jz >= ZW moves down by ZS rows and jx >= XW right by XS columns,
// so that the two halo strips of one axis form one set.  Cell k of the set
// goes to thread k % NT, pass k / NT (NT threads per block).  load() issues
// every pass's loads before store() combines them, so a thread's loads are
// all in flight at once.
template <int NT, int ZL, int NZ, int XL, int NX, int ZW = 0, int ZS = 0, int XW = 0, int XS = 0>
struct CellsT {
    static constexpr int N = NZ * NX;
    static constexpr int IT = (N + NT - 1) / NT;
    __device__ static __forceinline__ void cell(int t, int& lz, int& lx) {
        const int e = threadIdx.x + NT * t;
        const int jz = e % NZ, jx = e / NZ;
        lz = ZL + jz + ((ZS != 0 && jz >= ZW) ? ZS : 0);
        lx = XL + jx + ((XS != 0 && jx >= XW) ? XS : 0);
        // past the end of the set: a row far outside every grid, so that the
        // load goes to the clamped address (a line every block reads) rather
        // than to a node of another tile
        if (N % NT != 0 && e >= N) lz = -(1 << 20);
    }
    // ld(lz, lx, vals) issues the K loads of a cell from addresses that are
    // valid for any (lz, lx) (clamped outside the grid): passes past the end
    // of the set load too but store nothing.
    template <int K, typename LD>
    __device__ static __forceinline__ void load(LD ld, float (&v)[IT][K]) {
#pragma unroll
        for (int t = 0; t < IT; ++t) {
            int lz, lx;
            cell(t, lz, lx);
            ld(lz, lx, v[t]);
        }
    }
    // st(lz, lx, vals) combines the values and writes the cell's LDS entry.
    template <int K, typename ST>
    __device__ static __forceinline__ void store(ST st, float (&v)[IT][K]) {
#pragma unroll
        for (int t = 0; t < IT; ++t) {
            if (N % NT != 0 && threadIdx.x + NT * t >= N) continue;
            int lz, lx;
            cell(t, lz, lx);
            st(lz, lx, v[t]);
        }
    }
};
// Blocks of NTHREADS threads (every 2D kernel).
template <int ZL, int NZ, int XL, int NX, int ZW = 0, int ZS = 0, int XW = 0, int XS = 0>
using Cells = CellsT<NTHREADS, ZL, NZ, XL, NX, ZW, ZS, XW, XS>;

// Whether the CPML coefficients of index g (node or half node) on an axis
// of n nodes may be nonzero: the absorbing strips are the first npml and the
// last npml + 1 indices (the half node just outside the last interior node
// already lies in the strip).
__device__ __forceinline__ bool in_pml(int g, int n, int npml) { return g < npml || g >= n - npml - 1; }

// Forward staggered derivative at half node i + 1/2 from node values around
// LDS index c with stride s: sum_k c_k (f[i+k] - f[i-k+1]).
__device__ __forceinline__ float d_half(const float* f, int c, int s, const float* ck) {
    float r = ck[0] * (f[c + s] - f[c]);
    r = fmaf(ck[1], f[c + 2 * s] - f[c - s], r);
    r = fmaf(ck[2], f[c + 3 * s] - f[c - 2 * s], r);
    r = fmaf(ck[3], f[c + 4 * s] - f[c - 3 * s], r);
    return r;
}

// Backward staggered derivative at node i from half-node values (g[j] at
// j + 1/2): sum_k c_k (g[i+k-1] - g[i-k]).
__device__ __forceinline__ float d_node(const float* g, int c, int s, const float* ck) {
    float r = ck[0] * (g[c] - g[c - s]);
    r = fmaf(ck[1], g[c + s] - g[c - 2 * s], r);
    r = fmaf(ck[2], g[c + 2 * s] - g[c - 3 * s], r);
    r = fmaf(ck[3], g[c + 3 * s] - g[c - 4 * s], r);
    return r;
}

}  // namespace lsrtm
