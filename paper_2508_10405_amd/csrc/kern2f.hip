// Fused 2D time steps: one kernel per step instead of a velocity and a
// pressure phase (and one adjoint kernel instead of two).
//
// A tile of BZ x BX nodes stages the pressure of the previous step on a cross
// with a 7-node halo, computes the new velocities on the tile plus the 4-node
// halo the pressure update needs (redundantly with the neighbouring tiles),
// keeps them in LDS and then updates the pressure of the tile.  Every field
// that a tile reads at halo nodes is double-buffered (read "cur", write
// "next", roles swapped every step), so no tile overwrites a value another
// tile still reads; the background phi (read only at its own node) is
// updated in place, the scattered/adjoint phi is double-buffered like the
// rest because the adjoint reads it at halo nodes.
// Each expression is the one of the two-phase kernels (kern2d.hip) with the
// same operation order (the adjoint on the same scaled state Q = -dt kappa p~,
// U_a = -dt b_a v~_a), so both schedules give identical bits.  Algorithmic
// HBM traffic per node and step: 64 B (Born; two-phase 88), 44 B (replay;
// 56), 64 B (adjoint; 72).
#include "common.h"
#include "kernels.h"

namespace lsrtm {

template <int BZ, int BX>
struct F2 {
    static constexpr int PZ = BZ + 14;        // cross rows -7 .. BZ+6
    static constexpr int PX = BX + 14;        // cross cols -7 .. BX+6
    static constexpr int NPL = PZ * PX;
    static constexpr int VZ = BZ + 7;         // velocity rows -4 .. BZ+2
    static constexpr int VX = BX + 7;         // velocity cols -4 .. BX+2
    static constexpr int NVZ = VZ * BX;
    static constexpr int NVX = BZ * VX;
    static constexpr int NP = BZ * BX;
    static constexpr int R = NP / NTHREADS;
    static_assert(NP % NTHREADS == 0, "tile must hold a multiple of 256 nodes");
};

// ---------------------------------------------------------------------------
// Forward step: background (+ scattered for BORN, + replay store for SEG)
// ---------------------------------------------------------------------------
template <int BZ, int BX, bool BORN, bool SEG>
__global__ void __launch_bounds__(NTHREADS)
k2f_step(const DSlot* __restrict__ slots, const int4* __restrict__ tiles, Coef C, int n, int sstep, int flag, TileRec tr)
{
    using T = F2<BZ, BX>;
    constexpr int R = T::R;
    constexpr int K = BORN ? 2 : 1;
    using CZ = Cells<-7, BZ + 14, 0, BX>;            // p on the tile columns, rows -7 .. BZ+6
    using CX = Cells<0, BZ, -7, 14, 0, 0, 7, BX>;    // p on cols -7 .. -1 and BX .. BX+6
    __shared__ float sp[T::NPL];
    __shared__ float sq[BORN ? T::NPL : 1];
    __shared__ float svz[T::NVZ];
    __shared__ float svx[T::NVX];
    __shared__ float swz[BORN ? T::NVZ : 1];
    __shared__ float swx[BORN ? T::NVX : 1];
    const int tix = xcd_remap(blockIdx.x, gridDim.x);
    const int4 tl = tiles[tix];
    const DSlot& S = slots[tl.x];
    const int z0 = tl.y, x0 = tl.z;
    const int nz = S.n[0], nx = S.n[1], npml = S.npml;
    const long long ldz = S.ldz;
    // Every global load before the first barrier, from addresses that are
    // valid for any cell (element 0 where a cell is outside the grid or a
    // CPML memory is not needed outside the strips).
    // pointwise loads of the pressure update
    float kk[R], lk[R], ph0[R], ph1[R], et0[R], et1[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = threadIdx.x + NTHREADS * r;
        const int gz = z0 + e % BZ, gx = x0 + e / BZ;
        const bool in = gz < nz && gx < nx;
        const long long i = in ? gx * ldz + gz : 0;
        const long long iz = in && in_pml(gz, nz, npml) ? i : 0;
        const long long ix = in && in_pml(gx, nx, npml) ? i : 0;
        kk[r] = S.kdt[i];
        ph0[r] = S.phi[0][iz];
        ph1[r] = S.phi[1][ix];
        if (BORN) {
            lk[r] = S.dlnk[i];
            et0[r] = S.eta[0][iz];
            et1[r] = S.eta[1][ix];
        }
    }
    // velocity regions: v_z on rows -4 .. BZ+2 of the tile columns, v_x on
    // cols -4 .. BX+2 of the tile rows, with their pointwise inputs
    constexpr int NZR = BZ + 7, NXR = BZ;
    constexpr int RZ = (T::NVZ + NTHREADS - 1) / NTHREADS;
    constexpr int RX = (T::NVX + NTHREADS - 1) / NTHREADS;
    float zv[RZ], zb[RZ], zb1[RZ], zw[RZ], zr0[RZ], zr1[RZ], zps[RZ], zxs[RZ];
    float xv[RX], xb[RX], xb1[RX], xw[RX], xr0[RX], xr1[RX], xps[RX], xxs[RX];
#pragma unroll
    for (int t = 0; t < RZ; ++t) {
        const int e = threadIdx.x + NTHREADS * t;
        const int lz = -4 + e % NZR, lx = e / NZR;
        const int gz = z0 + lz, gx = x0 + lx;
        const bool in = e < T::NVZ && (unsigned)gz < (unsigned)nz && gx < nx;
        const long long i = in ? gx * ldz + gz : 0;
        const long long im = in && in_pml(gz, nz, npml) ? i : 0;
        zv[t] = S.v[0][i];
        zb[t] = S.sb[i];   // dt b_z = sb here times sb at the upper z-neighbour
        zb1[t] = S.sb[(in && gz + 1 < nz) ? i + 1 : i];
        zps[t] = S.psi[0][im];
        if (BORN) {
            zw[t] = S.w[0][i];
            zr0[t] = S.dlnr[i];
            zr1[t] = S.dlnr[(in && gz + 1 < nz) ? i + 1 : i];
            zxs[t] = S.xi[0][im];
        }
    }
#pragma unroll
    for (int t = 0; t < RX; ++t) {
        const int e = threadIdx.x + NTHREADS * t;
        const int lz = e % NXR, lx = -4 + e / NXR;
        const int gz = z0 + lz, gx = x0 + lx;
        const bool in = e < T::NVX && gz < nz && (unsigned)gx < (unsigned)nx;
        const long long i = in ? gx * ldz + gz : 0;
        const long long im = in && in_pml(gx, nx, npml) ? i : 0;
        xv[t] = S.v[1][i];
        xb[t] = S.sb[i];
        xb1[t] = S.sb[(in && gx + 1 < nx) ? i + ldz : i];
        xps[t] = S.psi[1][im];
        if (BORN) {
            xw[t] = S.w[1][i];
            xr0[t] = S.dlnr[i];
            xr1[t] = S.dlnr[(in && gx + 1 < nx) ? i + ldz : i];
            xxs[t] = S.xi[1][im];
        }
    }
    // p (and dp) of the previous step on the cross
    auto inside = [&](int lz, int lx) {
        return (unsigned)(z0 + lz) < (unsigned)nz && (unsigned)(x0 + lx) < (unsigned)nx;
    };
    auto ldp = [&](int lz, int lx, float* v) {
        const long long i = inside(lz, lx) ? (x0 + lx) * ldz + (z0 + lz) : 0;
        v[0] = S.p[i];
        if (BORN) v[1] = S.q[i];
    };
    auto stp = [&](int lz, int lx, const float* v) {
        const bool in = inside(lz, lx);
        const int c = (lx + 7) * T::PZ + lz + 7;
        sp[c] = in ? v[0] : 0.f;
        if (BORN) sq[c] = in ? v[1] : 0.f;
    };
    float hz[CZ::IT][K], hx[CX::IT][K];
    CZ::load(ldp, hz);
    CX::load(ldp, hx);
    CZ::store(stp, hz);
    CX::store(stp, hx);
    __syncthreads();
    const gfloat* achz = S.cpml[0];
    const gfloat* bchz = S.cpml[0] + nz;
    const gfloat* achx = S.cpml[1];
    const gfloat* bchx = S.cpml[1] + nx;
    gfloat* __restrict__ seg = S.seg + (long long)sstep * 3 * S.npts;
#pragma unroll
    for (int t = 0; t < RZ; ++t) {
        const int e = threadIdx.x + NTHREADS * t;
        if (e >= T::NVZ) continue;
        const int lz = -4 + e % NZR, lx = e / NZR;
        const int gz = z0 + lz, gx = x0 + lx;
        const int cv = lx * T::VZ + lz + 4;
        if (!((unsigned)gz < (unsigned)nz && gx < nx)) {
            svz[cv] = 0.f;
            if (BORN) swz[cv] = 0.f;
            continue;
        }
        const bool own = lz >= 0 && lz < BZ;
        const long long i = gx * ldz + gz;
        const int c = (lx + 7) * T::PZ + lz + 7;
        const float az = achz[gz];
        const float bz = zb[t] * zb1[t];
        float g = d_half(sp, c, 1, C.c[0]);
        if (az != 0.f) {
            const float ps = fmaf(bchz[gz], zps[t], az * g);
            if (own) S.psin[0][i] = ps;
            g = g + ps;
        }
        const float dv = -bz * g;
        const float vn = zv[t] + dv;
        svz[cv] = vn;
        if (own) {
            S.vn[0][i] = vn;
            if (SEG) seg[i] = g;   // the gradient behind dv, for migration
        }
        if (BORN) {
            float gq = d_half(sq, c, 1, C.c[0]);
            if (az != 0.f) {
                const float ps = fmaf(bchz[gz], zxs[t], az * gq);
                if (own) S.xin[0][i] = ps;
                gq = gq + ps;
            }
            const float wn = (zw[t] - bz * gq) - 0.5f * (zr0[t] + zr1[t]) * dv;
            swz[cv] = wn;
            if (own) S.wn[0][i] = wn;
        }
    }
#pragma unroll
    for (int t = 0; t < RX; ++t) {
        const int e = threadIdx.x + NTHREADS * t;
        if (e >= T::NVX) continue;
        const int lz = e % NXR, lx = -4 + e / NXR;
        const int gz = z0 + lz, gx = x0 + lx;
        const int cv = (lx + 4) * BZ + lz;
        if (!(gz < nz && (unsigned)gx < (unsigned)nx)) {
            svx[cv] = 0.f;
            if (BORN) swx[cv] = 0.f;
            continue;
        }
        const bool own = lx >= 0 && lx < BX;
        const long long i = gx * ldz + gz;
        const int c = (lx + 7) * T::PZ + lz + 7;
        const float ax = achx[gx];
        const float bx = xb[t] * xb1[t];
        float g = d_half(sp, c, T::PZ, C.c[1]);
        if (ax != 0.f) {
            const float ps = fmaf(bchx[gx], xps[t], ax * g);
            if (own) S.psin[1][i] = ps;
            g = g + ps;
        }
        const float dv = -bx * g;
        const float vn = xv[t] + dv;
        svx[cv] = vn;
        if (own) {
            S.vn[1][i] = vn;
            if (SEG) seg[S.npts + i] = g;
        }
        if (BORN) {
            float gq = d_half(sq, c, T::PZ, C.c[1]);
            if (ax != 0.f) {
                const float ps = fmaf(bchx[gx], xxs[t], ax * gq);
                if (own) S.xin[1][i] = ps;
                gq = gq + ps;
            }
            const float wn = (xw[t] - bx * gq) - 0.5f * (xr0[t] + xr1[t]) * dv;
            swx[cv] = wn;
            if (own) S.wn[1][i] = wn;
        }
    }
    __syncthreads();
    // pressure of the tile
    const gfloat* aciz = S.cpml[0] + 2 * nz;
    const gfloat* bciz = S.cpml[0] + 3 * nz;
    const gfloat* acix = S.cpml[1] + 2 * nx;
    const gfloat* bcix = S.cpml[1] + 3 * nx;
    const float amp = S.src >= 0 ? S.src_amp[n] : 0.f;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = threadIdx.x + NTHREADS * r;
        const int lz = e % BZ, lx = e / BZ;
        const int gz = z0 + lz, gx = x0 + lx;
        if (gz >= nz || gx >= nx) continue;
        const long long i = gx * ldz + gz;
        const int cz = lx * T::VZ + lz + 4;
        const int cx = (lx + 4) * BZ + lz;
        const int cp = (lx + 7) * T::PZ + lz + 7;
        const float az = aciz[gz], ax = acix[gx];
        float ez = d_node(svz, cz, 1, C.c[0]);
        float ex = d_node(svx, cx, BZ, C.c[1]);
        if (az != 0.f) {
            const float ph = fmaf(bciz[gz], ph0[r], az * ez);
            S.phi[0][i] = ph;
            ez = ez + ph;
        }
        if (ax != 0.f) {
            const float ph = fmaf(bcix[gx], ph1[r], ax * ex);
            S.phi[1][i] = ph;
            ex = ex + ph;
        }
        const float q = ez + ex;
        const float k = kk[r];
        float pn = sp[cp] - k * q;
        if (i == S.src) pn = pn + amp;
        S.pn[i] = pn;
        if (SEG) seg[2 * S.npts + i] = q;
        if (!BORN && tr.d) tile_gather(tr, tix, e, n, pn);
        if (BORN) {
            float fz = d_node(swz, cz, 1, C.c[0]);
            float fx = d_node(swx, cx, BZ, C.c[1]);
            if (az != 0.f) {
                const float ph = fmaf(bciz[gz], et0[r], az * fz);
                S.etan[0][i] = ph;
                fz = fz + ph;
            }
            if (ax != 0.f) {
                const float ph = fmaf(bcix[gx], et1[r], ax * fx);
                S.etan[1][i] = ph;
                fx = fx + ph;
            }
            const float dq = fz + fx;
            const float qn = (sq[cp] - k * dq) + lk[r] * (-k * q);
            S.qn[i] = qn;
            if (tr.d) tile_gather(tr, tix, e, n, qn);
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoint step (transpose of the forward step): phase A on the tile plus the
// velocity halo, then phase B on the tile.  flag = 1 on the first reverse
// step (no pending update of chi).
// ---------------------------------------------------------------------------
template <int BZ, int BX>
__global__ void __launch_bounds__(NTHREADS)
k2f_adj(const DSlot* __restrict__ slots, const int4* __restrict__ tiles, Coef C, int n, int sstep, int flag, TileRec tr)
{
    using T = F2<BZ, BX>;
    constexpr int R = T::R;
    using CZ = Cells<-7, BZ + 14, 0, BX>;      // e~_z rows -7 .. BZ+6 of the tile columns
    using CX = Cells<0, BZ, -7, BX + 14>;      // e~_x cols -7 .. BX+6 of the tile rows
    __shared__ float sez[(BZ + 14) * BX];
    __shared__ float sex[BZ * (BX + 14)];
    __shared__ float sgz[T::NVZ];             // g~_z rows -4 .. BZ+2
    __shared__ float sgx[T::NVX];             // g~_x cols -4 .. BX+2
    __shared__ float sxz[T::NVZ];             // -dv_z v~_z (lnrho imaging)
    __shared__ float sxx[T::NVX];
    const int tix = xcd_remap(blockIdx.x, gridDim.x);
    const int4 tl = tiles[tix];
    const DSlot& S = slots[tl.x];
    const int z0 = tl.y, x0 = tl.z;
    const int nz = S.n[0], nx = S.n[1], npml = S.npml;
    const long long ldz = S.ldz;
    const gfloat* __restrict__ segz = S.seg + (long long)sstep * 3 * S.npts;
    const gfloat* __restrict__ segx = segz + S.npts;
    const gfloat* __restrict__ segq = segz + 2 * S.npts;
    // Every global load before the first barrier (clamped addresses, as in
    // the forward step).
    float pt[R], kk[R], gk[R], qn[R], gr[R], et0[R], et1[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = threadIdx.x + NTHREADS * r;
        const int gz = z0 + e % BZ, gx = x0 + e / BZ;
        const bool in = gz < nz && gx < nx;
        const long long i = in ? gx * ldz + gz : 0;
        pt[r] = S.q[i];   // Q = -dt kappa p~
        kk[r] = S.kdt[i];
        gk[r] = S.gk[i];
        qn[r] = segq[i];
        gr[r] = S.gr[i];
        et0[r] = S.eta[0][in && in_pml(gz, nz, npml) ? i : 0];
        et1[r] = S.eta[1][in && in_pml(gx, nx, npml) ? i : 0];
    }
    const gfloat* aciz = S.cpml[0] + 2 * nz;
    const gfloat* bciz = S.cpml[0] + 3 * nz;
    const gfloat* acix = S.cpml[1] + 2 * nx;
    const gfloat* bcix = S.cpml[1] + 3 * nx;
    // velocity regions (as in the forward step) with their pointwise inputs
    constexpr int NZR = BZ + 7, NXR = BZ;
    constexpr int RZ = (T::NVZ + NTHREADS - 1) / NTHREADS;
    constexpr int RX = (T::NVX + NTHREADS - 1) / NTHREADS;
    float zv[RZ], zb[RZ], zs[RZ], zc[RZ], xv[RX], xb[RX], xs[RX], xc[RX];
#pragma unroll
    for (int t = 0; t < RZ; ++t) {
        const int e = threadIdx.x + NTHREADS * t;
        const int lz = -4 + e % NZR, lx = e / NZR;
        const int gz = z0 + lz, gx = x0 + lx;
        const bool in = e < T::NVZ && (unsigned)gz < (unsigned)nz && gx < nx;
        const long long i = in ? gx * ldz + gz : 0;
        zv[t] = S.w[0][i];
        zb[t] = S.bdt[0][i];
        zs[t] = segz[i];
        zc[t] = S.xi[0][in && in_pml(gz, nz, npml) ? i : 0];
    }
#pragma unroll
    for (int t = 0; t < RX; ++t) {
        const int e = threadIdx.x + NTHREADS * t;
        const int lz = e % NXR, lx = -4 + e / NXR;
        const int gz = z0 + lz, gx = x0 + lx;
        const bool in = e < T::NVX && gz < nz && (unsigned)gx < (unsigned)nx;
        const long long i = in ? gx * ldz + gz : 0;
        xv[t] = S.w[1][i];
        xb[t] = S.bdt[1][i];
        xs[t] = segx[i];
        xc[t] = S.xi[1][in && in_pml(gx, nx, npml) ? i : 0];
    }
    // e~_a on the crosses: Q, the CPML coefficient and phi~
    auto inside = [&](int lz, int lx) {
        return (unsigned)(z0 + lz) < (unsigned)nz && (unsigned)(x0 + lx) < (unsigned)nx;
    };
    auto lde_z = [&](int lz, int lx, float* v) {
        const int gz = z0 + lz, gx = x0 + lx;
        const bool in = inside(lz, lx);
        const long long i = in ? gx * ldz + gz : 0;
        v[0] = S.q[i];
        v[1] = aciz[in ? gz : 0];
        v[2] = S.eta[0][in && in_pml(gz, nz, npml) ? i : 0];
    };
    auto lde_x = [&](int lz, int lx, float* v) {
        const int gz = z0 + lz, gx = x0 + lx;
        const bool in = inside(lz, lx);
        const long long i = in ? gx * ldz + gz : 0;
        v[0] = S.q[i];
        v[1] = acix[in ? gx : 0];
        v[2] = S.eta[1][in && in_pml(gx, nx, npml) ? i : 0];
    };
    auto ete = [&](bool in, const float* v) {
        float e = 0.f;
        if (in) {
            const float qt = v[0];
            const float a = v[1];
            e = a != 0.f ? qt + a * (v[2] + qt) : qt;
        }
        return e;
    };
    float hz[CZ::IT][3], hx[CX::IT][3];
    CZ::load(lde_z, hz);
    CX::load(lde_x, hx);
    CZ::store([&](int lz, int lx, const float* v) { sez[lx * (BZ + 14) + lz + 7] = ete(inside(lz, lx), v); }, hz);
    CX::store([&](int lz, int lx, const float* v) { sex[(lx + 7) * BZ + lz] = ete(inside(lz, lx), v); }, hx);
    __syncthreads();
    const gfloat* achz = S.cpml[0];
    const gfloat* bchz = S.cpml[0] + nz;
    const gfloat* achx = S.cpml[1];
    const gfloat* bchx = S.cpml[1] + nx;
    // phase A for v~_z on rows -4 .. BZ+2, then g~_z and the imaging term
#pragma unroll
    for (int t = 0; t < RZ; ++t) {
        const int e = threadIdx.x + NTHREADS * t;
        if (e >= T::NVZ) continue;
        const int lz = -4 + e % NZR, lx = e / NZR;
        const int gz = z0 + lz, gx = x0 + lx;
        const int cv = lx * T::VZ + lz + 4;
        if (!((unsigned)gz < (unsigned)nz && gx < nx)) {
            sgz[cv] = 0.f;
            sxz[cv] = 0.f;
            continue;
        }
        const bool own = lz >= 0 && lz < BZ;
        const long long i = gx * ldz + gz;
        const float vo = zv[t];
        const float b = zb[t];
        const float a = achz[gz];
        float chi = 0.f;
        if (a != 0.f) {
            chi = zc[t];
            if (!flag) chi = bchz[gz] * (chi + vo);
            if (own) S.xin[0][i] = chi;
        }
        const float vn = vo + b * d_half(sez, lx * (BZ + 14) + lz + 7, 1, C.c[0]);
        if (own) S.wn[0][i] = vn;
        const float h = vn;
        sgz[cv] = a != 0.f ? h + a * (chi + h) : h;
        sxz[cv] = -zs[t] * vn;
    }
#pragma unroll
    for (int t = 0; t < RX; ++t) {
        const int e = threadIdx.x + NTHREADS * t;
        if (e >= T::NVX) continue;
        const int lz = e % NXR, lx = -4 + e / NXR;
        const int gz = z0 + lz, gx = x0 + lx;
        const int cv = (lx + 4) * BZ + lz;
        if (!(gz < nz && (unsigned)gx < (unsigned)nx)) {
            sgx[cv] = 0.f;
            sxx[cv] = 0.f;
            continue;
        }
        const bool own = lx >= 0 && lx < BX;
        const long long i = gx * ldz + gz;
        const float vo = xv[t];
        const float b = xb[t];
        const float a = achx[gx];
        float chi = 0.f;
        if (a != 0.f) {
            chi = xc[t];
            if (!flag) chi = bchx[gx] * (chi + vo);
            if (own) S.xin[1][i] = chi;
        }
        const float vn = vo + b * d_half(sex, (lx + 7) * BZ + lz, BZ, C.c[1]);
        if (own) S.wn[1][i] = vn;
        const float h = vn;
        sgx[cv] = a != 0.f ? h + a * (chi + h) : h;
        sxx[cv] = -xs[t] * vn;
    }
    __syncthreads();
    // phase B on the tile
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = threadIdx.x + NTHREADS * r;
        const int lz = e % BZ, lx = e / BZ;
        const int gz = z0 + lz, gx = x0 + lx;
        if (gz >= nz || gx >= nx) continue;
        const long long i = gx * ldz + gz;
        const int cz = lx * T::VZ + lz + 4;
        const int cx = (lx + 4) * BZ + lz;
        const float az = aciz[gz], ax = acix[gx];
        if (az != 0.f) S.etan[0][i] = bciz[gz] * (et0[r] + pt[r]);
        if (ax != 0.f) S.etan[1][i] = bcix[gx] * (et1[r] + pt[r]);
        S.gk[i] = gk[r] + qn[r] * pt[r];
        const float xz1 = gz > 0 ? sxz[cz - 1] : 0.f;
        const float xx1 = gx > 0 ? sxx[cx - BZ] : 0.f;
        // the last node of an axis also takes the other half of its own
        // product (transpose of the clamped forward average)
        const float tz = 0.5f * (sxz[cz] + xz1) + (gz + 1 == nz ? 0.5f * sxz[cz] : 0.f);
        const float tx = 0.5f * (sxx[cx] + xx1) + (gx + 1 == nx ? 0.5f * sxx[cx] : 0.f);
        S.gr[i] = gr[r] + (tz + tx);
        const float dz = d_node(sgz, cz, 1, C.c[0]);
        const float dx = d_node(sgx, cx, BZ, C.c[1]);
        float qn_ = pt[r] + kk[r] * (dz + dx);
        if (tr.y && n > 0) qn_ = qn_ - kk[r] * tile_inject(tr, tix, e, n - 1);
        S.qn[i] = qn_;
    }
}

// ---------------------------------------------------------------------------
template <int BZ, int BX>
static hipError_t launch2f_t(int kind, int ntiles, hipStream_t st, const Slot* slots,
                             const int4* tiles, const Coef& C, int n, int sstep, int flag, const TileRec& tr,
                            hipEvent_t e0, hipEvent_t e1)
{
    dim3 g(ntiles), b(NTHREADS);
    const DSlot* ds = dev_slots(slots);
    switch (kind) {
    case K_BG_V:   launch_k(k2f_step<BZ, BX, false, false>, g, b, st, e0, e1, ds, tiles, C, n, sstep, flag, tr); break;
    case K_SEG_V:  launch_k(k2f_step<BZ, BX, false, true>, g, b, st, e0, e1, ds, tiles, C, n, sstep, flag, tr); break;
    case K_BORN_V: launch_k(k2f_step<BZ, BX, true, false>, g, b, st, e0, e1, ds, tiles, C, n, sstep, flag, tr); break;
    case K_ADJ_A:  launch_k(k2f_adj<BZ, BX>, g, b, st, e0, e1, ds, tiles, C, n, sstep, flag, tr); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Fused schedule: kind is the velocity-phase kind of the step (K_BG_V,
// K_SEG_V, K_BORN_V) or K_ADJ_A for the adjoint step.
hipError_t launch2f(int kind, int tile_id, int ntiles, hipStream_t st, const Slot* slots,
                    const int4* tiles, const Coef& C, int n, int sstep, int flag, const TileRec& tr,
                            hipEvent_t e0, hipEvent_t e1)
{
    if (ntiles <= 0) return hipSuccess;
    switch (tile_id) {
    case 0: return launch2f_t<32, 8>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, tr, e0, e1);
    case 1: return launch2f_t<32, 16>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, tr, e0, e1);
    case 2: return launch2f_t<32, 32>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, tr, e0, e1);
    case 3: return launch2f_t<64, 4>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, tr, e0, e1);
    case 4: return launch2f_t<64, 8>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, tr, e0, e1);
    case 5: return launch2f_t<64, 16>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, tr, e0, e1);
    case 6: return launch2f_t<128, 4>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, tr, e0, e1);
    case 7: return launch2f_t<128, 8>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, tr, e0, e1);
    case 8: return launch2f_t<256, 4>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, tr, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace lsrtm
