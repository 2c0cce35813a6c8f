// 3D stencil kernels of the velocity-pressure propagator (gfx950).
//
// A tile t = (slot, z0, x0, y0 | y1 << 16) covers BZ x BX nodes of a (z, x)
// plane and marches through planes y0 .. y1 - 1 along y.  The z- and x-derivatives of the current
// plane come from an LDS tile with the 4-node halo each derivative needs; the
// y-derivative comes from a queue of the eight neighbouring planes kept in
// registers, so every value of the staged field is read from memory once per
// march.  The halos hold exactly the cells a derivative reads (three on one
// side, four on the other).  A tile of 128 rows or more that spans the whole
// padded z extent (256 rows in blocks of 1024 threads, one column per four
// waves, on a grid of up to 256 padded rows) has no z-halo at all: its halo
// rows lie outside the grid and stay zero.  Arrays read at a node's
// upper neighbours (sb for dt b_a, dlnrho for the density source) are read
// once per plane: the next plane's values are carried in registers and the
// z+1 and x+1 neighbours come from LDS, so that no line of them is fetched
// twice.  On every plane a thread issues all of its global loads at once --
// the queue's new front, the arrays it reads pointwise, the CPML memories of
// its nodes and its share of the halo -- from addresses that are always valid
// (element 0 of the array, or of the plane, where a value lies outside the
// grid or outside the absorbing strips), so no branch separates them; values
// are combined and written to LDS only after that.  The z and x CPML
// coefficients of a thread's nodes are read once, before the march.  The
// phases and the CPML bookkeeping are those of the 2D kernels (section 2 of
// the paper for V/P, eq. scattereqln for the Born sources, appendix A for the
// adjoint phases A/B), the adjoint state scaled as there (Q = -dt kappa p~,
// U_a = -dt b_a v~_a); the replay buffer holds G_a p + psi_a for the three
// axes and q per step.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace lsrtm {

template <int BZ, int BX, int NT>
struct Tile3 {
    static constexpr int LZ = BZ + 2 * HW;
    static constexpr int LX = BX + 2 * HW;
    static constexpr int NL = LZ * LX;
    static constexpr int NP = BZ * BX;
    static constexpr int R = NP / NT;
    static constexpr int LB = (BZ + 1) * (BX + 1);   // a plane of sb or dlnrho with the upper neighbours
    static_assert(NP % NT == 0, "tile must hold a multiple of the block's threads");
};

// Loads and stores of a shot's arrays that a launch touches at a node's own
// position only (each value read once and written once): non-temporal, so
// that they do not evict from L2 the lines of the staged fields, which
// neighbouring tiles read again as halos.  The model arrays (dt kappa, sb,
// dlnrho, dlnkappa) are shared by every shot on the same window and keep
// ordinary loads: the other shots of a launch read them again.
__device__ __forceinline__ float ldo(const gfloat* a, unsigned i) { return __builtin_nontemporal_load(&elem(a, i)); }
__device__ __forceinline__ void sto(gfloat* a, unsigned i, float v) { __builtin_nontemporal_store(v, &elem(a, i)); }

// Whether a tile spans the whole padded z extent: its z-halo then lies
// outside the grid on both sides and is zero.
template <int BZ>
__device__ __forceinline__ bool tile3_zfull(const DSlot* __restrict__ slots, const int4* __restrict__ tiles) {
    const int4 tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    return tl.y == 0 && slots[tl.x].n[0] <= BZ;
}

// The upper neighbours of a tile's nodes that lie outside the tile: column
// BX (rows 0 .. BZ-1) and, unless the tile spans the whole z extent, row BZ
// (columns 0 .. BX-1).  Cell k goes to thread k % NT, pass k / NT; cell()
// tells whether the pass holds a cell.  Passes past the end get a row far
// outside the grid, so they load the clamped address and store nothing.
template <int NT, int BZ, int BX, bool ZF>
struct Edge {
    static constexpr int N = BZ + (ZF ? 0 : BX);
    static constexpr int IT = (N + NT - 1) / NT;
    __device__ static __forceinline__ bool cell(int t, int& lz, int& lx) {
        const int k = threadIdx.x + NT * t;
        lz = k < BZ ? k : k < N ? BZ : -(1 << 20);
        lx = k < BZ ? BX : k - BZ;
        return k < N;
    }
};

// Zero rows -HW .. -1 and BZ .. BZ+HW-1 of the tile columns of an LDS tile
// (outside the grid on a tile that spans the whole z extent).
template <int NT, int BZ, int BX>
__device__ __forceinline__ void zero_zhalo(float* s) {
    constexpr int LZ = BZ + 2 * HW;
    for (int k = threadIdx.x; k < 2 * HW * BX; k += NT) {
        const int j = k % (2 * HW), lx = HW + k / (2 * HW);
        s[lx * LZ + (j < HW ? j : BZ + j)] = 0.f;
    }
}

// A tile (slot, z0, x0, y0 | y1 << 16) marches through planes y0 .. y1 - 1.
__device__ __forceinline__ int tile3_y0(const int4& t) { return t.w & 0xffff; }
__device__ __forceinline__ int tile3_y1(const int4& t) { return (int)((unsigned)t.w >> 16); }

// Whether a tile, with the halo planes and cells its queues and staging
// read, reaches a CPML strip.  The tiles that do not skip every CPML
// coefficient and memory load (the coefficients are zero there); each kernel
// branches once, on entry, between two instantiations of its tile body, so
// neither holds a branch between its loads.
template <int BZ, int BX>
__device__ __forceinline__ bool tile3_pml(const DSlot* __restrict__ slots, const int4* __restrict__ tiles) {
    const int4 tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const DSlot& S = slots[tl.x];
    const int z0 = tl.y, x0 = tl.z, y0 = tile3_y0(tl), y1 = tile3_y1(tl);
    const int nz = S.n[0], nx = S.n[1], ny = S.n[2], npml = S.npml;
    return z0 - HW - 1 < npml || z0 + BZ + HW >= nz - npml - 1 ||
           x0 - HW - 1 < npml || x0 + BX + HW >= nx - npml - 1 ||
           y0 - HW - 1 < npml || y1 + HW >= ny - npml - 1;
}

// y-derivative from a queue Q[m] = f(y + m - off): the staggered difference
// sum_k c_k (Q[3+k] - Q[4-k]) is G_y (off = 3) or D_y (off = 4).
__device__ __forceinline__ float d_queue(const float* Q, const float* ck) {
    float r = ck[0] * (Q[4] - Q[3]);
    r = fmaf(ck[1], Q[5] - Q[2], r);
    r = fmaf(ck[2], Q[6] - Q[1], r);
    r = fmaf(ck[3], Q[7] - Q[0], r);
    return r;
}

#define TILE3_SETUP                                                           \
    using T = Tile3<BZ, BX, NT>;                                              \
    constexpr int R = T::R;                                                   \
    const int4 tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];                  \
    const DSlot& S = slots[tl.x];                                             \
    const int z0 = tl.y, x0 = tl.z, y0 = tile3_y0(tl), y1 = tile3_y1(tl);     \
    const int nz = S.n[0], nx = S.n[1], ny = S.n[2], npml = S.npml;           \
    const unsigned sx = (unsigned)S.sx, sy = (unsigned)S.sy;                  \
    int lzr[R], lxr[R];                                                       \
    bool ok[R], pz[R], px[R];                                                 \
    unsigned ib[R];                                                           \
    _Pragma("unroll") for (int r = 0; r < R; ++r) {                           \
        const int e = threadIdx.x + NT * r;                                   \
        lzr[r] = e % BZ;                                                      \
        lxr[r] = e / BZ;                                                      \
        ok[r] = z0 + lzr[r] < nz && x0 + lxr[r] < nx;                         \
        ib[r] = ok[r] ? (x0 + lxr[r]) * sx + (z0 + lzr[r]) : 0;               \
        pz[r] = PML && ok[r] && in_pml(z0 + lzr[r], nz, npml);                \
        px[r] = PML && ok[r] && in_pml(x0 + lxr[r], nx, npml);                \
    }                                                                         \
    /* CPML coefficient or memory: zero on tiles away from the strips */      \
    auto cp = [&](const gfloat* a, unsigned j) -> float {                    \
        return PML ? elem(a, j) : 0.f;                                        \
    };                                                                        \
    /* a CPML memory at the node's own position (read once) */                \
    auto cpo = [&](const gfloat* a, unsigned j) -> float {                   \
        return PML ? ldo(a, j) : 0.f;                                         \
    };                                                                        \
    auto inside = [&](int lz, int lx) {                                       \
        return (unsigned)(z0 + lz - HW) < (unsigned)nz &&                     \
               (unsigned)(x0 + lx - HW) < (unsigned)nx;                       \
    };                                                                        \
    /* index of LDS cell (lz, lx) on plane offset py, element py outside */   \
    auto cidx = [&](int lz, int lx, unsigned py) -> unsigned {                \
        return (inside(lz, lx) ? (x0 + lx - HW) * sx + (z0 + lz - HW) : 0) + py; \
    };                                                                        \
    /* index of node (z0 + lz, x0 + lx) on plane offset py, py outside */     \
    auto nidx = [&](int lz, int lx, unsigned py) -> unsigned {                \
        return ((unsigned)(z0 + lz) < (unsigned)nz &&                         \
                (unsigned)(x0 + lx) < (unsigned)nx ? (x0 + lx) * sx + (z0 + lz) : 0) + py; \
    };                                                                        \
    /* value of f at node r of plane y, zero outside the grid */              \
    auto at = [&](const gfloat* f, int r, int y) -> float {                   \
        const bool v = ok[r] && (unsigned)y < (unsigned)ny;                   \
        const float x = elem(f, v ? ib[r] + y * sy : 0u);                     \
        return v ? x : 0.f;                                                   \
    };                                                                        \
    /* the same for an array read at own positions only */                   \
    auto ato = [&](const gfloat* f, int r, int y) -> float {                  \
        const bool v = ok[r] && (unsigned)y < (unsigned)ny;                   \
        const float x = ldo(f, v ? ib[r] + y * sy : 0u);                      \
        return v ? x : 0.f;                                                   \
    };

// ---------------------------------------------------------------------------
// V phase
// ---------------------------------------------------------------------------
template <int BZ, int BX, int NT, bool BORN, bool SEG, bool PML, bool ZF>
__device__ __forceinline__ void
v3_tile(const DSlot* __restrict__ slots, const int4* __restrict__ tiles, const Coef& C, int n, int sstep, int flag,
        float* __restrict__ sp, float* __restrict__ sq, float* __restrict__ lsb, float* __restrict__ ldr)
{
    TILE3_SETUP
    constexpr int K = BORN ? 2 : 1;
    // G_a at the half node i + 1/2 reads nodes i - 3 .. i + 4
    using CZ = CellsT<NT, 1, 2 * HW - 1, HW, BX, HW - 1, BZ>;         // rows -3 .. -1 and BZ .. BZ+3
    using CX = CellsT<NT, HW, BZ, 1, 2 * HW - 1, 0, 0, HW - 1, BX>;   // columns -3 .. -1 and BX .. BX+3
    using CE = Edge<NT, BZ, BX, ZF>;
    float Qp[R][8], Qq[R][8];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            Qp[r][m + 1] = at(S.p, r, y0 - 3 + m);
            if (BORN) Qq[r][m + 1] = at(S.q, r, y0 - 3 + m);
        }
    const gfloat* achz = S.cpml[0];
    const gfloat* bchz = S.cpml[0] + nz;
    const gfloat* achx = S.cpml[1];
    const gfloat* bchx = S.cpml[1] + nx;
    const gfloat* achy = S.cpml[2];
    const gfloat* bchy = S.cpml[2] + ny;
    // the z and x CPML coefficients of a node are the same on every plane
    float achz_[R], bchz_[R], achx_[R], bchx_[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int gz = ok[r] ? z0 + lzr[r] : 0, gx = ok[r] ? x0 + lxr[r] : 0;
        achz_[r] = cp(achz, gz);
        bchz_[r] = cp(bchz, gz);
        achx_[r] = cp(achx, gx);
        bchx_[r] = cp(bchx, gx);
    }
    gfloat* __restrict__ seg = S.seg + (long long)sstep * 4 * S.npts;
    // dt b_a = sb at the node times sb at its upper neighbour along a.  sb
    // and dlnrho of the current plane (s0, r0) were read as the previous
    // plane's y-neighbours; their z+1 and x+1 neighbours come from LDS
    float s0[R], r0[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        s0[r] = elem(S.sb, ib[r] + y0 * sy);
        if (BORN) r0[r] = elem(S.dlnr, ib[r] + y0 * sy);
    }
    if constexpr (ZF) {
        zero_zhalo<NT, BZ, BX>(sp);
        if (BORN) zero_zhalo<NT, BZ, BX>(sq);
    }
    for (int y = y0; y < y1; ++y) {
        const unsigned py = y * sy;
        const bool py_ = PML && in_pml(y, ny, npml);
        float vz[R], vx[R], vy[R], sn[R], rn[R], wz[R], wx[R], wy[R];
        float m0[R], m1[R], m2[R], n0[R], n1[R], n2[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int m = 0; m < 7; ++m) {
                Qp[r][m] = Qp[r][m + 1];
                if (BORN) Qq[r][m] = Qq[r][m + 1];
            }
            Qp[r][7] = at(S.p, r, y + 4);
            if (BORN) Qq[r][7] = at(S.q, r, y + 4);
            const unsigned i = ib[r] + py;
            vz[r] = ldo(S.v[0], i);
            vx[r] = ldo(S.v[1], i);
            vy[r] = ldo(S.v[2], i);
            sn[r] = elem(S.sb, y + 1 < ny ? i + sy : i);
            m0[r] = cpo(S.psi[0], pz[r] ? i : 0);
            m1[r] = cpo(S.psi[1], px[r] ? i : 0);
            m2[r] = cpo(S.psi[2], ok[r] && py_ ? i : 0);
            if (BORN) {
                wz[r] = ldo(S.w[0], i);
                wx[r] = ldo(S.w[1], i);
                wy[r] = ldo(S.w[2], i);
                rn[r] = elem(S.dlnr, y + 1 < ny ? i + sy : i);
                n0[r] = cpo(S.xi[0], pz[r] ? i : 0);
                n1[r] = cpo(S.xi[1], px[r] ? i : 0);
                n2[r] = cpo(S.xi[2], ok[r] && py_ ? i : 0);
            }
        }
        auto ld = [&](int lz, int lx, float* v) {
            const unsigned i = cidx(lz, lx, py);
            v[0] = elem(S.p, i);
            if (BORN) v[1] = elem(S.q, i);
        };
        auto st = [&](int lz, int lx, const float* v) {
            const int c = lx * T::LZ + lz;
            const bool in = inside(lz, lx);
            sp[c] = in ? v[0] : 0.f;
            if (BORN) sq[c] = in ? v[1] : 0.f;
        };
        float hz[CZ::IT][K], hx[CX::IT][K], he[CE::IT][K];
        if constexpr (!ZF) CZ::load(ld, hz);
        CX::load(ld, hx);
#pragma unroll
        for (int t = 0; t < CE::IT; ++t) {
            int lz, lx;
            CE::cell(t, lz, lx);
            const unsigned j = nidx(lz, lx, py);
            he[t][0] = elem(S.sb, j);
            if (BORN) he[t][1] = elem(S.dlnr, j);
        }
        __syncthreads();   // the previous plane's LDS tile is no longer read
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int c = (lxr[r] + HW) * T::LZ + lzr[r] + HW;
            sp[c] = Qp[r][3];
            if (BORN) sq[c] = Qq[r][3];
            lsb[lxr[r] * (BZ + 1) + lzr[r]] = s0[r];
            if (BORN) ldr[lxr[r] * (BZ + 1) + lzr[r]] = r0[r];
        }
        if constexpr (!ZF) CZ::store(st, hz);
        CX::store(st, hx);
#pragma unroll
        for (int t = 0; t < CE::IT; ++t) {
            int lz, lx;
            if (CE::cell(t, lz, lx)) {
                lsb[lx * (BZ + 1) + lz] = he[t][0];
                if (BORN) ldr[lx * (BZ + 1) + lz] = he[t][1];
            }
        }
        __syncthreads();
        const float ay = cp(achy, y);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!ok[r]) continue;
            const int gz = z0 + lzr[r], gx = x0 + lxr[r];
            const unsigned i = ib[r] + py;
            const int c = (lxr[r] + HW) * T::LZ + lzr[r] + HW;
            const int e = lxr[r] * (BZ + 1) + lzr[r];
            const float az = achz_[r], ax = achx_[r];
            float gzp = d_half(sp, c, 1, C.c[0]);
            float gxp = d_half(sp, c, T::LZ, C.c[1]);
            float gyp = d_queue(Qp[r], C.c[2]);
            if (az != 0.f) {
                const float ps = fmaf(bchz_[r], m0[r], az * gzp);
                sto(S.psi[0], i, ps);
                gzp = gzp + ps;
            }
            if (ax != 0.f) {
                const float ps = fmaf(bchx_[r], m1[r], ax * gxp);
                sto(S.psi[1], i, ps);
                gxp = gxp + ps;
            }
            if (ay != 0.f) {
                const float ps = fmaf(elem(bchy, y), m2[r], ay * gyp);
                sto(S.psi[2], i, ps);
                gyp = gyp + ps;
            }
            // the last node of an axis takes its own value as the upper neighbour
            const float s1z = gz + 1 < nz ? lsb[e + 1] : s0[r];
            const float s1x = gx + 1 < nx ? lsb[e + BZ + 1] : s0[r];
            const float bz = s0[r] * s1z, bx = s0[r] * s1x, by = s0[r] * sn[r];
            const float dvz = -bz * gzp;
            const float dvx = -bx * gxp;
            const float dvy = -by * gyp;
            sto(S.v[0], i, vz[r] + dvz);
            sto(S.v[1], i, vx[r] + dvx);
            sto(S.v[2], i, vy[r] + dvy);
            if (SEG) {   // read back only k steps later: streaming stores
                __builtin_nontemporal_store(gzp, &elem(seg, i));
                __builtin_nontemporal_store(gxp, &elem(seg, S.npts + i));
                __builtin_nontemporal_store(gyp, &elem(seg, 2 * S.npts + i));
            }
            if (!BORN && !SEG && (flag & PH_ACCUMULATE)) {   // pseudo-Hessian: sum of dv_a^2
                elem(S.w[0], i) = elem(S.w[0], i) + dvz * dvz;
                elem(S.w[1], i) = elem(S.w[1], i) + dvx * dvx;
                elem(S.w[2], i) = elem(S.w[2], i) + dvy * dvy;
            }
            if (BORN) {
                float gzq = d_half(sq, c, 1, C.c[0]);
                float gxq = d_half(sq, c, T::LZ, C.c[1]);
                float gyq = d_queue(Qq[r], C.c[2]);
                if (az != 0.f) {
                    const float ps = fmaf(bchz_[r], n0[r], az * gzq);
                    sto(S.xi[0], i, ps);
                    gzq = gzq + ps;
                }
                if (ax != 0.f) {
                    const float ps = fmaf(bchx_[r], n1[r], ax * gxq);
                    sto(S.xi[1], i, ps);
                    gxq = gxq + ps;
                }
                if (ay != 0.f) {
                    const float ps = fmaf(elem(bchy, y), n2[r], ay * gyq);
                    sto(S.xi[2], i, ps);
                    gyq = gyq + ps;
                }
                const float r1z = gz + 1 < nz ? ldr[e + 1] : r0[r];
                const float r1x = gx + 1 < nx ? ldr[e + BZ + 1] : r0[r];
                sto(S.w[0], i, (wz[r] - bz * gzq) - 0.5f * (r0[r] + r1z) * dvz);
                sto(S.w[1], i, (wx[r] - bx * gxq) - 0.5f * (r0[r] + r1x) * dvx);
                sto(S.w[2], i, (wy[r] - by * gyq) - 0.5f * (r0[r] + rn[r]) * dvy);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            s0[r] = sn[r];
            if (BORN) r0[r] = rn[r];
        }
    }
}

// Runs body(pml, zf) with compile-time flags: whether the tile does CPML
// work (tile3_pml) and whether it spans the whole z extent (tiles of at
// least 128 rows; shorter ones always take the body with a z-halo).
template <int BZ, int BX, typename F>
__device__ __forceinline__ void tile3_dispatch(const DSlot* __restrict__ slots, const int4* __restrict__ tiles,
                                               F body) {
    const bool pml = tile3_pml<BZ, BX>(slots, tiles);
    if constexpr (BZ >= 128) {
        if (tile3_zfull<BZ>(slots, tiles)) {
            if (pml) body(std::true_type{}, std::true_type{});
            else body(std::false_type{}, std::true_type{});
            return;
        }
    }
    if (pml) body(std::true_type{}, std::false_type{});
    else body(std::false_type{}, std::false_type{});
}

template <int BZ, int BX, int NT, bool BORN, bool SEG>
__global__ void __launch_bounds__(NT)
k3_v(const DSlot* __restrict__ slots, const int4* __restrict__ tiles, Coef C, int n, int sstep, int flag)
{
    using T = Tile3<BZ, BX, NT>;
    __shared__ float sp[T::NL];
    __shared__ float sq[BORN ? T::NL : 1];
    __shared__ float lsb[T::LB];
    __shared__ float ldr[BORN ? T::LB : 1];
    tile3_dispatch<BZ, BX>(slots, tiles, [&](auto pml, auto zf) {
        v3_tile<BZ, BX, NT, BORN, SEG, decltype(pml)::value, decltype(zf)::value>(
            slots, tiles, C, n, sstep, flag, sp, sq, lsb, ldr);
    });
}

// ---------------------------------------------------------------------------
// P phase
// ---------------------------------------------------------------------------
template <int BZ, int BX, int NT, bool BORN, bool SEG, bool PML, bool ZF>
__device__ __forceinline__ void
p3_tile(const DSlot* __restrict__ slots, const int4* __restrict__ tiles, const Coef& C, int n, int sstep, int flag,
        float* __restrict__ svz, float* __restrict__ svx, float* __restrict__ swz, float* __restrict__ swx)
{
    TILE3_SETUP
    constexpr int K = BORN ? 2 : 1;
    // D_a at node i reads half nodes i - 4 .. i + 3: v_z (and w_z) on rows
    // -4 .. BZ+2 (the tile rows alone when the z-halo lies outside the grid),
    // v_x (and w_x) on columns -4 .. BX+2
    using CZ = std::conditional_t<ZF, CellsT<NT, HW, BZ, HW, BX>, CellsT<NT, 0, T::LZ - 1, HW, BX>>;
    using CX = CellsT<NT, HW, BZ, 0, T::LX - 1>;
    if constexpr (ZF) {
        zero_zhalo<NT, BZ, BX>(svz);
        if (BORN) zero_zhalo<NT, BZ, BX>(swz);
    }
    float Qv[R][8], Qw[R][8];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            Qv[r][m + 1] = ato(S.v[2], r, y0 - 4 + m);
            if (BORN) Qw[r][m + 1] = ato(S.w[2], r, y0 - 4 + m);
        }
    const gfloat* aciz = S.cpml[0] + 2 * nz;
    const gfloat* bciz = S.cpml[0] + 3 * nz;
    const gfloat* acix = S.cpml[1] + 2 * nx;
    const gfloat* bcix = S.cpml[1] + 3 * nx;
    const gfloat* aciy = S.cpml[2] + 2 * ny;
    const gfloat* bciy = S.cpml[2] + 3 * ny;
    // the z and x CPML coefficients of a node are the same on every plane
    float aciz_[R], bciz_[R], acix_[R], bcix_[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int gz = ok[r] ? z0 + lzr[r] : 0, gx = ok[r] ? x0 + lxr[r] : 0;
        aciz_[r] = cp(aciz, gz);
        bciz_[r] = cp(bciz, gz);
        acix_[r] = cp(acix, gx);
        bcix_[r] = cp(bcix, gx);
    }
    const float amp = S.src >= 0 ? elem(S.src_amp, n) : 0.f;
    gfloat* __restrict__ seg = S.seg + (long long)sstep * 4 * S.npts + 3 * S.npts;
    for (int y = y0; y < y1; ++y) {
        const unsigned py = y * sy;
        const bool py_ = PML && in_pml(y, ny, npml);
        float pp[R], kk[R], qq[R], lk[R], m0[R], m1[R], m2[R], n0[R], n1[R], n2[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int m = 0; m < 7; ++m) {
                Qv[r][m] = Qv[r][m + 1];
                if (BORN) Qw[r][m] = Qw[r][m + 1];
            }
            Qv[r][7] = ato(S.v[2], r, y + 3);
            if (BORN) Qw[r][7] = ato(S.w[2], r, y + 3);
            const unsigned i = ib[r] + py;
            pp[r] = ldo(S.p, i);
            kk[r] = elem(S.kdt, i);
            m0[r] = cpo(S.phi[0], pz[r] ? i : 0);
            m1[r] = cpo(S.phi[1], px[r] ? i : 0);
            m2[r] = cpo(S.phi[2], ok[r] && py_ ? i : 0);
            if (BORN) {
                qq[r] = ldo(S.q, i);
                lk[r] = elem(S.dlnk, i);
                n0[r] = cpo(S.eta[0], pz[r] ? i : 0);
                n1[r] = cpo(S.eta[1], px[r] ? i : 0);
                n2[r] = cpo(S.eta[2], ok[r] && py_ ? i : 0);
            }
        }
        float hz[CZ::IT][K], hx[CX::IT][K];
        CZ::load([&](int lz, int lx, float* v) {
            const unsigned i = cidx(lz, lx, py);
            v[0] = elem(S.v[0], i);
            if (BORN) v[1] = elem(S.w[0], i);
        }, hz);
        CX::load([&](int lz, int lx, float* v) {
            const unsigned i = cidx(lz, lx, py);
            v[0] = elem(S.v[1], i);
            if (BORN) v[1] = elem(S.w[1], i);
        }, hx);
        __syncthreads();
        CZ::store([&](int lz, int lx, const float* v) {
            const int c = lx * T::LZ + lz;
            const bool in = inside(lz, lx);
            svz[c] = in ? v[0] : 0.f;
            if (BORN) swz[c] = in ? v[1] : 0.f;
        }, hz);
        CX::store([&](int lz, int lx, const float* v) {
            const int c = lx * T::LZ + lz;
            const bool in = inside(lz, lx);
            svx[c] = in ? v[0] : 0.f;
            if (BORN) swx[c] = in ? v[1] : 0.f;
        }, hx);
        __syncthreads();
        const float ay = cp(aciy, y);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!ok[r]) continue;
            const int gz = z0 + lzr[r], gx = x0 + lxr[r];
            const unsigned i = ib[r] + py;
            const int c = (lxr[r] + HW) * T::LZ + lzr[r] + HW;
            const float az = aciz_[r], ax = acix_[r];
            float ez = d_node(svz, c, 1, C.c[0]);
            float ex = d_node(svx, c, T::LZ, C.c[1]);
            float ey = d_queue(Qv[r], C.c[2]);
            if (az != 0.f) {
                const float ph = fmaf(bciz_[r], m0[r], az * ez);
                sto(S.phi[0], i, ph);
                ez = ez + ph;
            }
            if (ax != 0.f) {
                const float ph = fmaf(bcix_[r], m1[r], ax * ex);
                sto(S.phi[1], i, ph);
                ex = ex + ph;
            }
            if (ay != 0.f) {
                const float ph = fmaf(elem(bciy, y), m2[r], ay * ey);
                sto(S.phi[2], i, ph);
                ey = ey + ph;
            }
            const float q = (ez + ex) + ey;
            const float k = kk[r];
            float pn = pp[r] - k * q;
            if (i == S.src) pn = pn + amp;
            sto(S.p, i, pn);
            if (SEG) __builtin_nontemporal_store(q, &elem(seg, i));
            if (!BORN && !SEG && (flag & PH_ACCUMULATE)) elem(S.gk, i) = elem(S.gk, i) + q * q;   // pseudo-Hessian
            if (BORN) {
                float fz = d_node(swz, c, 1, C.c[0]);
                float fx = d_node(swx, c, T::LZ, C.c[1]);
                float fy = d_queue(Qw[r], C.c[2]);
                if (az != 0.f) {
                    const float ph = fmaf(bciz_[r], n0[r], az * fz);
                    sto(S.eta[0], i, ph);
                    fz = fz + ph;
                }
                if (ax != 0.f) {
                    const float ph = fmaf(bcix_[r], n1[r], ax * fx);
                    sto(S.eta[1], i, ph);
                    fx = fx + ph;
                }
                if (ay != 0.f) {
                    const float ph = fmaf(elem(bciy, y), n2[r], ay * fy);
                    sto(S.eta[2], i, ph);
                    fy = fy + ph;
                }
                const float dq = (fz + fx) + fy;
                sto(S.q, i, (qq[r] - k * dq) + lk[r] * (-k * q));
            }
        }
    }
}

template <int BZ, int BX, int NT, bool BORN, bool SEG>
__global__ void __launch_bounds__(NT)
k3_p(const DSlot* __restrict__ slots, const int4* __restrict__ tiles, Coef C, int n, int sstep, int flag)
{
    using T = Tile3<BZ, BX, NT>;
    __shared__ float svz[T::NL];
    __shared__ float svx[T::NL];
    __shared__ float swz[BORN ? T::NL : 1];
    __shared__ float swx[BORN ? T::NL : 1];
    tile3_dispatch<BZ, BX>(slots, tiles, [&](auto pml, auto zf) {
        p3_tile<BZ, BX, NT, BORN, SEG, decltype(pml)::value, decltype(zf)::value>(
            slots, tiles, C, n, sstep, flag, svz, svx, swz, swx);
    });
}

// ---------------------------------------------------------------------------
// Adjoint phase A (transpose of P), as in the 2D kernels
// ---------------------------------------------------------------------------
template <int BZ, int BX, int NT, bool PML, bool ZF>
__device__ __forceinline__ void
a3_tile(const DSlot* __restrict__ slots, const int4* __restrict__ tiles, const Coef& C, int n, int sstep, int flag,
        float* __restrict__ sez, float* __restrict__ sex, float* __restrict__ lsb)
{
    TILE3_SETUP
    // the transposed G_a at half node i + 1/2 reads nodes i - 3 .. i + 4
    using CZ = CellsT<NT, 1, 2 * HW - 1, HW, BX, HW - 1, BZ>;         // rows -3 .. -1 and BZ .. BZ+3
    using CX = CellsT<NT, HW, BZ, 1, 2 * HW - 1, 0, 0, HW - 1, BX>;   // columns -3 .. -1 and BX .. BX+3
    using CE = Edge<NT, BZ, BX, ZF>;
    if constexpr (ZF) zero_zhalo<NT, BZ, BX>(sez);
    const gfloat* aciz = S.cpml[0] + 2 * nz;
    const gfloat* acix = S.cpml[1] + 2 * nx;
    const gfloat* aciy = S.cpml[2] + 2 * ny;
    const gfloat* achz = S.cpml[0];
    const gfloat* bchz = S.cpml[0] + nz;
    const gfloat* achx = S.cpml[1];
    const gfloat* bchx = S.cpml[1] + nx;
    const gfloat* achy = S.cpml[2];
    const gfloat* bchy = S.cpml[2] + ny;
    // the z and x CPML coefficients of a node are the same on every plane
    float aciz_[R], acix_[R], achz_[R], bchz_[R], achx_[R], bchx_[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int gz = ok[r] ? z0 + lzr[r] : 0, gx = ok[r] ? x0 + lxr[r] : 0;
        aciz_[r] = cp(aciz, gz);
        acix_[r] = cp(acix, gx);
        achz_[r] = cp(achz, gz);
        bchz_[r] = cp(bchz, gz);
        achx_[r] = cp(achx, gx);
        bchx_[r] = cp(bchx, gx);
    }
    const gfloat* __restrict__ segq = S.seg + (long long)sstep * 4 * S.npts + 3 * S.npts;
    // E[m] = e~_y(y + m - 3);  QT[m] = Q(y + m).  The loads of plane y are Q
    // and (inside the y-strips) phi~_y.
    float E[R][8], QT[R][5];
    auto front = [&](int r, int y, float& fq, float& fe) {
        const bool v = ok[r] && (unsigned)y < (unsigned)ny;
        const unsigned i = v ? ib[r] + y * sy : 0;
        fq = elem(S.q, i);
        fe = cpo(S.eta[2], v && in_pml(y, ny, npml) ? i : 0);
    };
    auto combine = [&](int r, int y, float fq, float fe, float& qt, float& ey) {
        const bool v = ok[r] && (unsigned)y < (unsigned)ny;
        qt = 0.f;
        ey = 0.f;
        if (v) {
            qt = fq;
            const float a = cp(aciy, y);
            ey = a != 0.f ? qt + a * (fe + qt) : qt;
        }
    };
#pragma unroll
    for (int r = 0; r < R; ++r) {
        float fq[7], fe[7];
#pragma unroll
        for (int m = 0; m < 7; ++m) front(r, y0 - 3 + m, fq[m], fe[m]);
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            float qt;
            combine(r, y0 - 3 + m, fq[m], fe[m], qt, E[r][m + 1]);
            if (m >= 3) QT[r][m - 2] = qt;
        }
    }
    // dt b_a of a node = sb there times sb at its upper neighbour.  sb of the
    // current plane (s0) was read as the previous plane's y-neighbour; its z+1
    // and x+1 neighbours come from LDS
    float s0[R];
#pragma unroll
    for (int r = 0; r < R; ++r) s0[r] = elem(S.sb, ib[r] + y0 * sy);
    // loads of e~ at a halo cell: the CPML coefficient, phi~, Q
    auto ldz_ = [&](int lz, int lx, unsigned py, float* v) {
        const int gz = z0 + lz - HW;
        const unsigned i = cidx(lz, lx, py);
        const bool in = inside(lz, lx);
        v[0] = cp(aciz, in ? gz : 0);
        v[1] = cp(S.eta[0], in && in_pml(gz, nz, npml) ? i : py);
        v[2] = elem(S.q, i);
    };
    auto ldx_ = [&](int lz, int lx, unsigned py, float* v) {
        const int gx = x0 + lx - HW;
        const unsigned i = cidx(lz, lx, py);
        const bool in = inside(lz, lx);
        v[0] = cp(acix, in ? gx : 0);
        v[1] = cp(S.eta[1], in && in_pml(gx, nx, npml) ? i : py);
        v[2] = elem(S.q, i);
    };
    auto ete = [&](bool in, const float* v) {
        float e = 0.f;
        if (in) {
            const float qt = v[2];
            e = v[0] != 0.f ? qt + v[0] * (v[1] + qt) : qt;
        }
        return e;
    };
    for (int y = y0; y < y1; ++y) {
        const unsigned py = y * sy;
        const bool py_ = PML && in_pml(y, ny, npml);
        float vz[R], vx[R], vy[R], gk[R], qn[R], e0[R], e1[R], fq[R], fe[R];
        float c0[R], c1[R], c2[R], sn[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            front(r, y + 4, fq[r], fe[r]);
            const unsigned i = ib[r] + py;
            vz[r] = ldo(S.w[0], i);
            vx[r] = ldo(S.w[1], i);
            vy[r] = ldo(S.w[2], i);
            gk[r] = ldo(S.gk, i);
            qn[r] = __builtin_nontemporal_load(&elem(segq, i));
            sn[r] = elem(S.sb, y + 1 < ny ? i + sy : i);
            e0[r] = cp(S.eta[0], pz[r] ? i : 0);
            e1[r] = cp(S.eta[1], px[r] ? i : 0);
            if (!flag) {
                const unsigned jz = pz[r] ? i : 0u, jx = px[r] ? i : 0u, jy = ok[r] && py_ ? i : 0u;
                c0[r] = cpo(S.xi[0], jz);
                c1[r] = cpo(S.xi[1], jx);
                c2[r] = cpo(S.xi[2], jy);
            }
        }
        float hz[CZ::IT][3], hx[CX::IT][3], he[CE::IT];
        if constexpr (!ZF) CZ::load([&](int lz, int lx, float* v) { ldz_(lz, lx, py, v); }, hz);
        CX::load([&](int lz, int lx, float* v) { ldx_(lz, lx, py, v); }, hx);
#pragma unroll
        for (int t = 0; t < CE::IT; ++t) {
            int lz, lx;
            CE::cell(t, lz, lx);
            he[t] = elem(S.sb, nidx(lz, lx, py));
        }
        __syncthreads();
        // interior from the queue, halos from memory
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int m = 0; m < 7; ++m) E[r][m] = E[r][m + 1];
#pragma unroll
            for (int m = 0; m < 4; ++m) QT[r][m] = QT[r][m + 1];
            combine(r, y + 4, fq[r], fe[r], QT[r][4], E[r][7]);
            const int c = (lxr[r] + HW) * T::LZ + lzr[r] + HW;
            const float qt = QT[r][0];
            float ez = qt, ex = qt;
            if (ok[r]) {
                const int gz = z0 + lzr[r], gx = x0 + lxr[r];
                const float az = aciz_[r], ax = acix_[r];
                if (az != 0.f) ez = qt + az * (e0[r] + qt);
                if (ax != 0.f) ex = qt + ax * (e1[r] + qt);
            }
            sez[c] = ez;
            sex[c] = ex;
            lsb[lxr[r] * (BZ + 1) + lzr[r]] = s0[r];
        }
        if constexpr (!ZF)
            CZ::store([&](int lz, int lx, const float* v) { sez[lx * T::LZ + lz] = ete(inside(lz, lx), v); }, hz);
        CX::store([&](int lz, int lx, const float* v) { sex[lx * T::LZ + lz] = ete(inside(lz, lx), v); }, hx);
#pragma unroll
        for (int t = 0; t < CE::IT; ++t) {
            int lz, lx;
            if (CE::cell(t, lz, lx)) lsb[lx * (BZ + 1) + lz] = he[t];
        }
        __syncthreads();
        const float hyc = cp(achy, y);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!ok[r]) continue;
            const int gz = z0 + lzr[r], gx = x0 + lxr[r];
            const unsigned i = ib[r] + py;
            const int c = (lxr[r] + HW) * T::LZ + lzr[r] + HW;
            if (!flag) {
                const float a = achz_[r], b = achx_[r];
                if (a != 0.f) sto(S.xi[0], i, bchz_[r] * (c0[r] + vz[r]));
                if (b != 0.f) sto(S.xi[1], i, bchx_[r] * (c1[r] + vx[r]));
                if (hyc != 0.f) sto(S.xi[2], i, elem(bchy, y) * (c2[r] + vy[r]));
            }
            sto(S.gk, i, gk[r] + qn[r] * QT[r][0]);
            const int e = lxr[r] * (BZ + 1) + lzr[r];
            const float s1z = gz + 1 < nz ? lsb[e + 1] : s0[r];
            const float s1x = gx + 1 < nx ? lsb[e + BZ + 1] : s0[r];
            const float bz = s0[r] * s1z, bx = s0[r] * s1x, by = s0[r] * sn[r];
            sto(S.w[0], i, vz[r] + bz * d_half(sez, c, 1, C.c[0]));
            sto(S.w[1], i, vx[r] + bx * d_half(sex, c, T::LZ, C.c[1]));
            sto(S.w[2], i, vy[r] + by * d_queue(E[r], C.c[2]));
        }
#pragma unroll
        for (int r = 0; r < R; ++r) s0[r] = sn[r];
    }
}

template <int BZ, int BX, int NT>
__global__ void __launch_bounds__(NT)
k3_a(const DSlot* __restrict__ slots, const int4* __restrict__ tiles, Coef C, int n, int sstep, int flag)
{
    using T = Tile3<BZ, BX, NT>;
    __shared__ float sez[T::NL];
    __shared__ float sex[T::NL];
    __shared__ float lsb[T::LB];
    tile3_dispatch<BZ, BX>(slots, tiles, [&](auto pml, auto zf) {
        a3_tile<BZ, BX, NT, decltype(pml)::value, decltype(zf)::value>(
            slots, tiles, C, n, sstep, flag, sez, sex, lsb);
    });
}

// ---------------------------------------------------------------------------
// Adjoint phase B (transpose of V), as in the 2D kernels; the products
// -(G_a p + psi_a) U_a of the lnrho image are formed while staging (z, x) or
// kept from the previous plane (y).
// ---------------------------------------------------------------------------
template <int BZ, int BX, int NT, bool PML, bool ZF>
__device__ __forceinline__ void
b3_tile(const DSlot* __restrict__ slots, const int4* __restrict__ tiles, const Coef& C, int n, int sstep, int flag,
        float* __restrict__ sgz, float* __restrict__ sgx, float* __restrict__ sxz, float* __restrict__ sxx)
{
    TILE3_SETUP
    // the transposed D_a at node i reads half nodes i - 4 .. i + 3 and the
    // lnrho product at i - 1: g~_z on rows -4 .. BZ+2 (the tile rows alone when
    // the z-halo lies outside the grid), g~_x on columns -4 .. BX+2
    using CZ = std::conditional_t<ZF, CellsT<NT, HW, BZ, HW, BX>, CellsT<NT, 0, T::LZ - 1, HW, BX>>;
    using CX = CellsT<NT, HW, BZ, 0, T::LX - 1>;
    if constexpr (ZF) {
        zero_zhalo<NT, BZ, BX>(sgz);
        zero_zhalo<NT, BZ, BX>(sxz);
    }
    const gfloat* achz = S.cpml[0];
    const gfloat* achx = S.cpml[1];
    const gfloat* achy = S.cpml[2];
    const gfloat* aciz = S.cpml[0] + 2 * nz;
    const gfloat* bciz = S.cpml[0] + 3 * nz;
    const gfloat* acix = S.cpml[1] + 2 * nx;
    const gfloat* bcix = S.cpml[1] + 3 * nx;
    const gfloat* aciy = S.cpml[2] + 2 * ny;
    const gfloat* bciy = S.cpml[2] + 3 * ny;
    // the z and x CPML coefficients of a node are the same on every plane
    float aciz_[R], bciz_[R], acix_[R], bcix_[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int gz = ok[r] ? z0 + lzr[r] : 0, gx = ok[r] ? x0 + lxr[r] : 0;
        aciz_[r] = cp(aciz, gz);
        bciz_[r] = cp(bciz, gz);
        acix_[r] = cp(acix, gx);
        bcix_[r] = cp(bcix, gx);
    }
    const gfloat* __restrict__ segz = S.seg + (long long)sstep * 4 * S.npts;
    const gfloat* __restrict__ segx = segz + S.npts;
    const gfloat* __restrict__ segy = segz + 2 * S.npts;
    // Gq[m] = g~_y(y + m - 4) from U_y and (inside the y-strips) chi_y;
    // Xp = -(G_y p + psi_y) U_y on the previous plane
    float Gq[R][8], Xp[R], Wq[R][4];
    auto front = [&](int r, int y, float* f) {
        const bool v = ok[r] && (unsigned)y < (unsigned)ny;
        const unsigned i = v ? ib[r] + y * sy : 0;
        f[0] = ldo(S.w[2], i);
        f[1] = cpo(S.xi[2], v && in_pml(y, ny, npml) ? i : 0);
    };
    auto gy_of = [&](int r, int y, const float* f) -> float {
        if (!(ok[r] && (unsigned)y < (unsigned)ny)) return 0.f;
        const float h = f[0];
        const float fc = f[1];
        const float a = cp(achy, y);
        return a != 0.f ? h + a * (fc + h) : h;
    };
#pragma unroll
    for (int r = 0; r < R; ++r) {
        float f[7][2];
#pragma unroll
        for (int m = 0; m < 7; ++m) front(r, y0 - 4 + m, f[m]);
        const bool pv = ok[r] && y0 > 0;
        const unsigned ip = pv ? ib[r] + (y0 - 1) * sy : 0u;
        const float s_ = elem(segy, ip), w_ = elem(S.w[2], ip);
#pragma unroll
        for (int m = 0; m < 7; ++m) Gq[r][m + 1] = gy_of(r, y0 - 4 + m, f[m]);
        Xp[r] = pv ? -s_ * w_ : 0.f;
        // Wq[k] = U_y(y + k): the queue's fronts, kept for the plane's own product
#pragma unroll
        for (int m = 0; m < 3; ++m) Wq[r][m + 1] = f[m + 4][0];
    }
    // loads of g~_a and of the image product at a cell: the CPML coefficient,
    // chi_a, U_a and G_a p + psi_a (on the rows / columns whose product is
    // needed)
    auto ldz_ = [&](int lz, int lx, unsigned py, float* v) {
        const int gz = z0 + lz - HW;
        const bool in = inside(lz, lx);
        const unsigned i = cidx(lz, lx, py);
        v[0] = cp(achz, in ? gz : 0);
        v[1] = cp(S.xi[0], in && in_pml(gz, nz, npml) ? i : py);
        v[2] = elem(S.w[0], i);
        v[3] = elem(segz, in && lz >= HW - 1 && lz < HW + BZ ? i : py);
    };
    auto ldx_ = [&](int lz, int lx, unsigned py, float* v) {
        const int gx = x0 + lx - HW;
        const bool in = inside(lz, lx);
        const unsigned i = cidx(lz, lx, py);
        v[0] = cp(achx, in ? gx : 0);
        v[1] = cp(S.xi[1], in && in_pml(gx, nx, npml) ? i : py);
        v[2] = elem(S.w[1], i);
        v[3] = elem(segx, in && lx >= HW - 1 && lx < HW + BX ? i : py);
    };
    for (int y = y0; y < y1; ++y) {
        const unsigned py = y * sy;
        const bool py_ = PML && in_pml(y, ny, npml);
        float pt[R], gr[R], sy_[R], kk[R], e0[R], e1[R], e2[R], fr[R][2];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            front(r, y + 3, fr[r]);
            const unsigned i = ib[r] + py;
            pt[r] = ldo(S.q, i);
            gr[r] = ldo(S.gr, i);
            sy_[r] = __builtin_nontemporal_load(&elem(segy, i));
            kk[r] = elem(S.kdt, i);
            e0[r] = cpo(S.eta[0], pz[r] ? i : 0);
            e1[r] = cpo(S.eta[1], px[r] ? i : 0);
            e2[r] = cpo(S.eta[2], ok[r] && py_ ? i : 0);
        }
        float hz[CZ::IT][4], hx[CX::IT][4];
        CZ::load([&](int lz, int lx, float* v) { ldz_(lz, lx, py, v); }, hz);
        CX::load([&](int lz, int lx, float* v) { ldx_(lz, lx, py, v); }, hx);
        __syncthreads();
        CZ::store([&](int lz, int lx, const float* v) {
            const int c = lx * T::LZ + lz;
            float g = 0.f, x = 0.f;
            if (inside(lz, lx)) {
                const float h = v[2];
                g = v[0] != 0.f ? h + v[0] * (v[1] + h) : h;
                if (lz >= HW - 1 && lz < HW + BZ) x = -v[3] * v[2];
            }
            sgz[c] = g;
            sxz[c] = x;
        }, hz);
        CX::store([&](int lz, int lx, const float* v) {
            const int c = lx * T::LZ + lz;
            float g = 0.f, x = 0.f;
            if (inside(lz, lx)) {
                const float h = v[2];
                g = v[0] != 0.f ? h + v[0] * (v[1] + h) : h;
                if (lx >= HW - 1 && lx < HW + BX) x = -v[3] * v[2];
            }
            sgx[c] = g;
            sxx[c] = x;
        }, hx);
        __syncthreads();
        const float ay = cp(aciy, y);
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int m = 0; m < 7; ++m) Gq[r][m] = Gq[r][m + 1];
            Gq[r][7] = gy_of(r, y + 3, fr[r]);
#pragma unroll
            for (int m = 0; m < 3; ++m) Wq[r][m] = Wq[r][m + 1];
            Wq[r][3] = fr[r][0];
            if (!ok[r]) continue;
            const int gz = z0 + lzr[r], gx = x0 + lxr[r];
            const unsigned i = ib[r] + py;
            const int c = (lxr[r] + HW) * T::LZ + lzr[r] + HW;
            const float az = aciz_[r], ax = acix_[r];
            if (az != 0.f) sto(S.eta[0], i, bciz_[r] * (e0[r] + pt[r]));
            if (ax != 0.f) sto(S.eta[1], i, bcix_[r] * (e1[r] + pt[r]));
            if (ay != 0.f) sto(S.eta[2], i, elem(bciy, y) * (e2[r] + pt[r]));
            const float xy0 = -sy_[r] * Wq[r][0];
            // the last node of an axis also takes the other half of its own
            // product (transpose of the clamped forward average)
            const float tz = 0.5f * (sxz[c] + sxz[c - 1]) + (gz + 1 == nz ? 0.5f * sxz[c] : 0.f);
            const float tx = 0.5f * (sxx[c] + sxx[c - T::LZ]) + (gx + 1 == nx ? 0.5f * sxx[c] : 0.f);
            const float ty = 0.5f * (xy0 + Xp[r]) + (y + 1 == ny ? 0.5f * xy0 : 0.f);
            sto(S.gr, i, gr[r] + ((tz + tx) + ty));
            Xp[r] = xy0;
            const float dz = d_node(sgz, c, 1, C.c[0]);
            const float dx = d_node(sgx, c, T::LZ, C.c[1]);
            const float dy = d_queue(Gq[r], C.c[2]);
            sto(S.q, i, pt[r] + kk[r] * ((dz + dx) + dy));
        }
    }
}

template <int BZ, int BX, int NT>
__global__ void __launch_bounds__(NT)
k3_b(const DSlot* __restrict__ slots, const int4* __restrict__ tiles, Coef C, int n, int sstep, int flag)
{
    using T = Tile3<BZ, BX, NT>;
    __shared__ float sgz[T::NL];
    __shared__ float sgx[T::NL];
    __shared__ float sxz[T::NL];
    __shared__ float sxx[T::NL];
    tile3_dispatch<BZ, BX>(slots, tiles, [&](auto pml, auto zf) {
        b3_tile<BZ, BX, NT, decltype(pml)::value, decltype(zf)::value>(
            slots, tiles, C, n, sstep, flag, sgz, sgx, sxz, sxx);
    });
}

// ---------------------------------------------------------------------------
template <int BZ, int BX, int NT>
static hipError_t launch3_t(int kind, int ntiles, hipStream_t st, const Slot* slots,
                            const int4* tiles, const Coef& C, int n, int sstep, int flag,
                            hipEvent_t e0, hipEvent_t e1)
{
    dim3 g(ntiles), b(NT);
    const DSlot* ds = dev_slots(slots);
    switch (kind) {
    case K_BG_V:    launch_k(k3_v<BZ, BX, NT, false, false>, g, b, st, e0, e1, ds, tiles, C, n, sstep, flag); break;
    case K_BG_P:    launch_k(k3_p<BZ, BX, NT, false, false>, g, b, st, e0, e1, ds, tiles, C, n, sstep, flag); break;
    case K_SEG_V:   launch_k(k3_v<BZ, BX, NT, false, true>, g, b, st, e0, e1, ds, tiles, C, n, sstep, flag); break;
    case K_SEG_P:   launch_k(k3_p<BZ, BX, NT, false, true>, g, b, st, e0, e1, ds, tiles, C, n, sstep, flag); break;
    case K_BORN_V:  launch_k(k3_v<BZ, BX, NT, true, false>, g, b, st, e0, e1, ds, tiles, C, n, sstep, flag); break;
    case K_BORN_P:  launch_k(k3_p<BZ, BX, NT, true, false>, g, b, st, e0, e1, ds, tiles, C, n, sstep, flag); break;
    case K_ADJ_A:   launch_k(k3_a<BZ, BX, NT>, g, b, st, e0, e1, ds, tiles, C, n, sstep, flag); break;
    case K_ADJ_B:   launch_k(k3_b<BZ, BX, NT>, g, b, st, e0, e1, ds, tiles, C, n, sstep, flag); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Tile shapes (z, x extents and the planes of a march).  Shapes 0-5 run in
// blocks of 256 threads, 9 and 10 in blocks of 512 (one node per thread);
// the tall shapes 6-8 in blocks of 1024 (one column of 256 rows per four
// waves, so a tile of 256 rows spans the whole padded z extent of grids up
// to 256 nodes deep).
const int kTiles3[][3] = {{64, 4, 32}, {64, 8, 32}, {64, 8, 64}, {32, 8, 64}, {128, 4, 64}, {64, 4, 64},
                          {256, 4, 32}, {256, 8, 32}, {128, 8, 32}, {64, 8, 32}, {128, 4, 32}};
const int kNumTiles3 = 11;

hipError_t launch3d(int kind, int tile_id, int ntiles, hipStream_t st, const Slot* slots,
                    const int4* tiles, const Coef& C, int n, int sstep, int flag,
                    hipEvent_t e0, hipEvent_t e1)
{
    if (ntiles <= 0) return hipSuccess;
    switch (tile_id) {
    case 0: case 5: return launch3_t<64, 4, 256>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, e0, e1);
    case 1: case 2: return launch3_t<64, 8, 256>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, e0, e1);
    case 3: return launch3_t<32, 8, 256>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, e0, e1);
    case 4: return launch3_t<128, 4, 256>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, e0, e1);
    case 6: return launch3_t<256, 4, 1024>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, e0, e1);
    case 7: return launch3_t<256, 8, 1024>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, e0, e1);
    case 8: return launch3_t<128, 8, 1024>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, e0, e1);
    case 9: return launch3_t<64, 8, 512>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, e0, e1);
    case 10: return launch3_t<128, 4, 512>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace lsrtm
