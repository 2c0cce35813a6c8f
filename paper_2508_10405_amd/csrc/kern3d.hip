// 3D stencil kernels of the velocity-pressure propagator (gfx950).
//
// A tile t = (slot, z0, x0, y0) covers BZ x BX nodes of a (z, x) plane and
// marches through BY planes along y.  The z- and x-derivatives of the current
// plane come from an LDS tile with the 4-node halo each derivative needs; the
// y-derivative comes from a queue of the eight neighbouring planes kept in
// registers, so every value of the staged field is read from memory once per
// march.  Arrays read pointwise are loaded before the LDS barrier of each
// plane.  The phases and the CPML bookkeeping are those of the 2D kernels
// (section 2 of the paper for V/P, eq. scattereqln for the Born sources,
// appendix A for the adjoint phases A/B); the replay buffer holds
// dv_z, dv_x, dv_y, q per step.
#include "common.h"
#include "kernels.h"

namespace lsrtm {

template <int BZ, int BX>
struct Tile3 {
    static constexpr int LZ = BZ + 2 * HW;
    static constexpr int LX = BX + 2 * HW;
    static constexpr int NL = LZ * LX;
    static constexpr int NP = BZ * BX;
    static constexpr int R = NP / NTHREADS;
    static_assert(NP % NTHREADS == 0, "tile must hold a multiple of 256 nodes");
};

template <int LZ, typename F>
__device__ __forceinline__ void region3(int zl, int zh, int xl, int xh, F f) {
    const int nzr = zh - zl, n = nzr * (xh - xl);
    for (int e = threadIdx.x; e < n; e += NTHREADS) {
        const int lz = zl + e % nzr, lx = xl + e / nzr;
        f(lz, lx, lx * LZ + lz);
    }
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
    using T = Tile3<BZ, BX>;                                                  \
    constexpr int R = T::R;                                                   \
    const int4 tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];                  \
    const DSlot& S = slots[tl.x];                                              \
    const int z0 = tl.y, x0 = tl.z, y0 = tl.w;                                \
    const int nz = S.n[0], nx = S.n[1], ny = S.n[2];                          \
    const long long sx = S.sx, sy = S.sy;                                     \
    const int y1 = y0 + BY < ny ? y0 + BY : ny;                               \
    int lzr[R], lxr[R];                                                       \
    bool ok[R];                                                               \
    long long ib[R];                                                          \
    _Pragma("unroll") for (int r = 0; r < R; ++r) {                           \
        const int e = threadIdx.x + NTHREADS * r;                             \
        lzr[r] = e % BZ;                                                      \
        lxr[r] = e / BZ;                                                      \
        ok[r] = z0 + lzr[r] < nz && x0 + lxr[r] < nx;                         \
        ib[r] = ok[r] ? (x0 + lxr[r]) * sx + (z0 + lzr[r]) : 0;               \
    }

// ---------------------------------------------------------------------------
// V phase
// ---------------------------------------------------------------------------
template <int BZ, int BX, int BY, bool BORN, bool SEG>
__global__ void __launch_bounds__(NTHREADS)
k3_v(const DSlot* __restrict__ slots, const int4* __restrict__ tiles, Coef C, int n, int sstep, int flag)
{
    TILE3_SETUP
    __shared__ float sp[T::NL];
    __shared__ float sq[BORN ? T::NL : 1];
    float Qp[R][8], Qq[R][8];
    auto at = [&](const gfloat* f, int r, int y) -> float {
        return (ok[r] && (unsigned)y < (unsigned)ny) ? f[ib[r] + y * sy] : 0.f;
    };
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
    gfloat* __restrict__ seg = S.seg + (long long)sstep * 4 * S.npts;
    for (int y = y0; y < y1; ++y) {
        const long long py = y * sy;
        float vz[R], vx[R], vy[R], bz[R], bx[R], by[R], wz[R], wx[R], wy[R], r0[R], r1z[R], r1x[R], r1y[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int m = 0; m < 7; ++m) {
                Qp[r][m] = Qp[r][m + 1];
                if (BORN) Qq[r][m] = Qq[r][m + 1];
            }
            Qp[r][7] = at(S.p, r, y + 4);
            if (BORN) Qq[r][7] = at(S.q, r, y + 4);
            const long long i = ib[r] + py;
            vz[r] = S.v[0][i];
            vx[r] = S.v[1][i];
            vy[r] = S.v[2][i];
            bz[r] = S.bdt[0][i];
            bx[r] = S.bdt[1][i];
            by[r] = S.bdt[2][i];
            if (BORN) {
                const int gz = z0 + lzr[r], gx = x0 + lxr[r];
                wz[r] = S.w[0][i];
                wx[r] = S.w[1][i];
                wy[r] = S.w[2][i];
                r0[r] = S.dlnr[i];
                r1z[r] = S.dlnr[gz + 1 < nz ? i + 1 : i];
                r1x[r] = S.dlnr[gx + 1 < nx ? i + sx : i];
                r1y[r] = S.dlnr[y + 1 < ny ? i + sy : i];
            }
        }
        __syncthreads();   // the previous plane's LDS tile is no longer read
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int c = (lxr[r] + HW) * T::LZ + lzr[r] + HW;
            sp[c] = Qp[r][3];
            if (BORN) sq[c] = Qq[r][3];
        }
        auto ld = [&](int lz, int lx, int c) {
            const int gz = z0 + lz - HW, gx = x0 + lx - HW;
            const bool in = (unsigned)gz < (unsigned)nz && (unsigned)gx < (unsigned)nx;
            const long long i = gx * sx + gz + py;
            sp[c] = in ? S.p[i] : 0.f;
            if (BORN) sq[c] = in ? S.q[i] : 0.f;
        };
        region3<T::LZ>(0, HW, HW, HW + BX, ld);
        region3<T::LZ>(HW + BZ, T::LZ, HW, HW + BX, ld);
        region3<T::LZ>(HW, HW + BZ, 0, HW, ld);
        region3<T::LZ>(HW, HW + BZ, HW + BX, T::LX, ld);
        __syncthreads();
        const float ay = achy[y];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!ok[r]) continue;
            const int gz = z0 + lzr[r], gx = x0 + lxr[r];
            const long long i = ib[r] + py;
            const int c = (lxr[r] + HW) * T::LZ + lzr[r] + HW;
            const float az = achz[gz], ax = achx[gx];
            float gzp = d_half(sp, c, 1, C.c[0]);
            float gxp = d_half(sp, c, T::LZ, C.c[1]);
            float gyp = d_queue(Qp[r], C.c[2]);
            if (az != 0.f) {
                const float ps = fmaf(bchz[gz], S.psi[0][i], az * gzp);
                S.psi[0][i] = ps;
                gzp = gzp + ps;
            }
            if (ax != 0.f) {
                const float ps = fmaf(bchx[gx], S.psi[1][i], ax * gxp);
                S.psi[1][i] = ps;
                gxp = gxp + ps;
            }
            if (ay != 0.f) {
                const float ps = fmaf(bchy[y], S.psi[2][i], ay * gyp);
                S.psi[2][i] = ps;
                gyp = gyp + ps;
            }
            const float dvz = -bz[r] * gzp;
            const float dvx = -bx[r] * gxp;
            const float dvy = -by[r] * gyp;
            S.v[0][i] = vz[r] + dvz;
            S.v[1][i] = vx[r] + dvx;
            S.v[2][i] = vy[r] + dvy;
            if (SEG) {
                seg[i] = dvz;
                seg[S.npts + i] = dvx;
                seg[2 * S.npts + i] = dvy;
            }
            if (BORN) {
                float gzq = d_half(sq, c, 1, C.c[0]);
                float gxq = d_half(sq, c, T::LZ, C.c[1]);
                float gyq = d_queue(Qq[r], C.c[2]);
                if (az != 0.f) {
                    const float ps = fmaf(bchz[gz], S.xi[0][i], az * gzq);
                    S.xi[0][i] = ps;
                    gzq = gzq + ps;
                }
                if (ax != 0.f) {
                    const float ps = fmaf(bchx[gx], S.xi[1][i], ax * gxq);
                    S.xi[1][i] = ps;
                    gxq = gxq + ps;
                }
                if (ay != 0.f) {
                    const float ps = fmaf(bchy[y], S.xi[2][i], ay * gyq);
                    S.xi[2][i] = ps;
                    gyq = gyq + ps;
                }
                S.w[0][i] = (wz[r] - bz[r] * gzq) - 0.5f * (r0[r] + r1z[r]) * dvz;
                S.w[1][i] = (wx[r] - bx[r] * gxq) - 0.5f * (r0[r] + r1x[r]) * dvx;
                S.w[2][i] = (wy[r] - by[r] * gyq) - 0.5f * (r0[r] + r1y[r]) * dvy;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// P phase
// ---------------------------------------------------------------------------
template <int BZ, int BX, int BY, bool BORN, bool SEG>
__global__ void __launch_bounds__(NTHREADS)
k3_p(const DSlot* __restrict__ slots, const int4* __restrict__ tiles, Coef C, int n, int sstep, int flag)
{
    TILE3_SETUP
    __shared__ float svz[T::NL];
    __shared__ float svx[T::NL];
    __shared__ float swz[BORN ? T::NL : 1];
    __shared__ float swx[BORN ? T::NL : 1];
    float Qv[R][8], Qw[R][8];
    auto at = [&](const gfloat* f, int r, int y) -> float {
        return (ok[r] && (unsigned)y < (unsigned)ny) ? f[ib[r] + y * sy] : 0.f;
    };
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            Qv[r][m + 1] = at(S.v[2], r, y0 - 4 + m);
            if (BORN) Qw[r][m + 1] = at(S.w[2], r, y0 - 4 + m);
        }
    const gfloat* aciz = S.cpml[0] + 2 * nz;
    const gfloat* bciz = S.cpml[0] + 3 * nz;
    const gfloat* acix = S.cpml[1] + 2 * nx;
    const gfloat* bcix = S.cpml[1] + 3 * nx;
    const gfloat* aciy = S.cpml[2] + 2 * ny;
    const gfloat* bciy = S.cpml[2] + 3 * ny;
    const float amp = S.src >= 0 ? S.src_amp[n] : 0.f;
    gfloat* __restrict__ seg = S.seg + (long long)sstep * 4 * S.npts + 3 * S.npts;
    for (int y = y0; y < y1; ++y) {
        const long long py = y * sy;
        float pp[R], kk[R], qq[R], lk[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int m = 0; m < 7; ++m) {
                Qv[r][m] = Qv[r][m + 1];
                if (BORN) Qw[r][m] = Qw[r][m + 1];
            }
            Qv[r][7] = at(S.v[2], r, y + 3);
            if (BORN) Qw[r][7] = at(S.w[2], r, y + 3);
            const long long i = ib[r] + py;
            pp[r] = S.p[i];
            kk[r] = S.kdt[i];
            if (BORN) {
                qq[r] = S.q[i];
                lk[r] = S.dlnk[i];
            }
        }
        __syncthreads();
        auto lz_ = [&](int lz, int lx, int c) {
            const int gz = z0 + lz - HW, gx = x0 + lx - HW;
            const bool in = (unsigned)gz < (unsigned)nz && (unsigned)gx < (unsigned)nx;
            const long long i = gx * sx + gz + py;
            svz[c] = in ? S.v[0][i] : 0.f;
            if (BORN) swz[c] = in ? S.w[0][i] : 0.f;
        };
        auto lx_ = [&](int lz, int lx, int c) {
            const int gz = z0 + lz - HW, gx = x0 + lx - HW;
            const bool in = (unsigned)gz < (unsigned)nz && (unsigned)gx < (unsigned)nx;
            const long long i = gx * sx + gz + py;
            svx[c] = in ? S.v[1][i] : 0.f;
            if (BORN) swx[c] = in ? S.w[1][i] : 0.f;
        };
        region3<T::LZ>(0, T::LZ, HW, HW + BX, lz_);
        region3<T::LZ>(HW, HW + BZ, 0, T::LX, lx_);
        __syncthreads();
        const float ay = aciy[y];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!ok[r]) continue;
            const int gz = z0 + lzr[r], gx = x0 + lxr[r];
            const long long i = ib[r] + py;
            const int c = (lxr[r] + HW) * T::LZ + lzr[r] + HW;
            const float az = aciz[gz], ax = acix[gx];
            float ez = d_node(svz, c, 1, C.c[0]);
            float ex = d_node(svx, c, T::LZ, C.c[1]);
            float ey = d_queue(Qv[r], C.c[2]);
            if (az != 0.f) {
                const float ph = fmaf(bciz[gz], S.phi[0][i], az * ez);
                S.phi[0][i] = ph;
                ez = ez + ph;
            }
            if (ax != 0.f) {
                const float ph = fmaf(bcix[gx], S.phi[1][i], ax * ex);
                S.phi[1][i] = ph;
                ex = ex + ph;
            }
            if (ay != 0.f) {
                const float ph = fmaf(bciy[y], S.phi[2][i], ay * ey);
                S.phi[2][i] = ph;
                ey = ey + ph;
            }
            const float q = (ez + ex) + ey;
            const float k = kk[r];
            float pn = pp[r] - k * q;
            if (i == S.src) pn = pn + amp;
            S.p[i] = pn;
            if (SEG) seg[i] = q;
            if (BORN) {
                float fz = d_node(swz, c, 1, C.c[0]);
                float fx = d_node(swx, c, T::LZ, C.c[1]);
                float fy = d_queue(Qw[r], C.c[2]);
                if (az != 0.f) {
                    const float ph = fmaf(bciz[gz], S.eta[0][i], az * fz);
                    S.eta[0][i] = ph;
                    fz = fz + ph;
                }
                if (ax != 0.f) {
                    const float ph = fmaf(bcix[gx], S.eta[1][i], ax * fx);
                    S.eta[1][i] = ph;
                    fx = fx + ph;
                }
                if (ay != 0.f) {
                    const float ph = fmaf(bciy[y], S.eta[2][i], ay * fy);
                    S.eta[2][i] = ph;
                    fy = fy + ph;
                }
                const float dq = (fz + fx) + fy;
                S.q[i] = (qq[r] - k * dq) + lk[r] * (-k * q);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoint phase A (transpose of P), see kern2d.hip
// ---------------------------------------------------------------------------
template <int BZ, int BX, int BY>
__global__ void __launch_bounds__(NTHREADS)
k3_a(const DSlot* __restrict__ slots, const int4* __restrict__ tiles, Coef C, int n, int sstep, int flag)
{
    TILE3_SETUP
    __shared__ float sez[T::NL];
    __shared__ float sex[T::NL];
    const gfloat* aciz = S.cpml[0] + 2 * nz;
    const gfloat* acix = S.cpml[1] + 2 * nx;
    const gfloat* aciy = S.cpml[2] + 2 * ny;
    const gfloat* achz = S.cpml[0];
    const gfloat* bchz = S.cpml[0] + nz;
    const gfloat* achx = S.cpml[1];
    const gfloat* bchx = S.cpml[1] + nx;
    const gfloat* achy = S.cpml[2];
    const gfloat* bchy = S.cpml[2] + ny;
    const gfloat* __restrict__ segq = S.seg + (long long)sstep * 4 * S.npts + 3 * S.npts;
    // E[m] = e~_y(y + m - 3);  QT[m] = q~(y + m), q~ = -dt kappa p~
    float E[R][8], QT[R][5];
    auto qt_at = [&](int r, int y) -> float {
        if (!ok[r] || (unsigned)y >= (unsigned)ny) return 0.f;
        const long long i = ib[r] + y * sy;
        return -S.kdt[i] * S.q[i];
    };
    auto ey_of = [&](int r, int y, float qt) -> float {
        if (!ok[r] || (unsigned)y >= (unsigned)ny) return 0.f;
        const float a = aciy[y];
        return a != 0.f ? qt + a * (S.eta[2][ib[r] + y * sy] + qt) : qt;
    };
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            const int yy = y0 - 3 + m;
            const float qt = qt_at(r, yy);
            E[r][m + 1] = ey_of(r, yy, qt);
            if (m >= 3) QT[r][m - 2] = qt;
        }
    for (int y = y0; y < y1; ++y) {
        const long long py = y * sy;
        float vz[R], vx[R], vy[R], gk[R], qn[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int m = 0; m < 7; ++m) E[r][m] = E[r][m + 1];
#pragma unroll
            for (int m = 0; m < 4; ++m) QT[r][m] = QT[r][m + 1];
            const float qt = qt_at(r, y + 4);
            QT[r][4] = qt;
            E[r][7] = ey_of(r, y + 4, qt);
            const long long i = ib[r] + py;
            vz[r] = S.w[0][i];
            vx[r] = S.w[1][i];
            vy[r] = S.w[2][i];
            gk[r] = S.gk[i];
            qn[r] = segq[i];
        }
        __syncthreads();
        // interior from the queue, halos from memory
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int c = (lxr[r] + HW) * T::LZ + lzr[r] + HW;
            const float qt = QT[r][0];
            float ez = qt, ex = qt;
            if (ok[r]) {
                const int gz = z0 + lzr[r], gx = x0 + lxr[r];
                const float az = aciz[gz], ax = acix[gx];
                if (az != 0.f) ez = qt + az * (S.eta[0][ib[r] + py] + qt);
                if (ax != 0.f) ex = qt + ax * (S.eta[1][ib[r] + py] + qt);
            }
            sez[c] = ez;
            sex[c] = ex;
        }
        auto hz = [&](int lz, int lx, int c) {
            const int gz = z0 + lz - HW, gx = x0 + lx - HW;
            float e = 0.f;
            if ((unsigned)gz < (unsigned)nz && (unsigned)gx < (unsigned)nx) {
                const long long i = gx * sx + gz + py;
                const float qt = -S.kdt[i] * S.q[i];
                const float a = aciz[gz];
                e = a != 0.f ? qt + a * (S.eta[0][i] + qt) : qt;
            }
            sez[c] = e;
        };
        auto hx = [&](int lz, int lx, int c) {
            const int gz = z0 + lz - HW, gx = x0 + lx - HW;
            float e = 0.f;
            if ((unsigned)gz < (unsigned)nz && (unsigned)gx < (unsigned)nx) {
                const long long i = gx * sx + gz + py;
                const float qt = -S.kdt[i] * S.q[i];
                const float a = acix[gx];
                e = a != 0.f ? qt + a * (S.eta[1][i] + qt) : qt;
            }
            sex[c] = e;
        };
        region3<T::LZ>(0, HW, HW, HW + BX, hz);
        region3<T::LZ>(HW + BZ, T::LZ, HW, HW + BX, hz);
        region3<T::LZ>(HW, HW + BZ, 0, HW, hx);
        region3<T::LZ>(HW, HW + BZ, HW + BX, T::LX, hx);
        __syncthreads();
        const float hyc = achy[y];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!ok[r]) continue;
            const int gz = z0 + lzr[r], gx = x0 + lxr[r];
            const long long i = ib[r] + py;
            const int c = (lxr[r] + HW) * T::LZ + lzr[r] + HW;
            if (!flag) {
                const float a = achz[gz], b = achx[gx];
                if (a != 0.f) S.xi[0][i] = bchz[gz] * (S.xi[0][i] + (-S.bdt[0][i] * vz[r]));
                if (b != 0.f) S.xi[1][i] = bchx[gx] * (S.xi[1][i] + (-S.bdt[1][i] * vx[r]));
                if (hyc != 0.f) S.xi[2][i] = bchy[y] * (S.xi[2][i] + (-S.bdt[2][i] * vy[r]));
            }
            S.gk[i] = gk[r] + qn[r] * QT[r][0];
            S.w[0][i] = vz[r] - d_half(sez, c, 1, C.c[0]);
            S.w[1][i] = vx[r] - d_half(sex, c, T::LZ, C.c[1]);
            S.w[2][i] = vy[r] - d_queue(E[r], C.c[2]);
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoint phase B (transpose of V), see kern2d.hip
// ---------------------------------------------------------------------------
template <int BZ, int BX, int BY>
__global__ void __launch_bounds__(NTHREADS)
k3_b(const DSlot* __restrict__ slots, const int4* __restrict__ tiles, Coef C, int n, int sstep, int flag)
{
    TILE3_SETUP
    __shared__ float sgz[T::NL];
    __shared__ float sgx[T::NL];
    const gfloat* achz = S.cpml[0];
    const gfloat* achx = S.cpml[1];
    const gfloat* achy = S.cpml[2];
    const gfloat* aciz = S.cpml[0] + 2 * nz;
    const gfloat* bciz = S.cpml[0] + 3 * nz;
    const gfloat* acix = S.cpml[1] + 2 * nx;
    const gfloat* bcix = S.cpml[1] + 3 * nx;
    const gfloat* aciy = S.cpml[2] + 2 * ny;
    const gfloat* bciy = S.cpml[2] + 3 * ny;
    const gfloat* __restrict__ segz = S.seg + (long long)sstep * 4 * S.npts;
    const gfloat* __restrict__ segx = segz + S.npts;
    const gfloat* __restrict__ segy = segz + 2 * S.npts;
    // Gq[m] = g~_y(y + m - 4);  Xp = -dv_y v~_y on the previous plane
    float Gq[R][8], Xp[R];
    auto gy_at = [&](int r, int y) -> float {
        if (!ok[r] || (unsigned)y >= (unsigned)ny) return 0.f;
        const long long i = ib[r] + y * sy;
        const float h = -S.bdt[2][i] * S.w[2][i];
        const float a = achy[y];
        return a != 0.f ? h + a * (S.xi[2][i] + h) : h;
    };
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int m = 0; m < 7; ++m) Gq[r][m + 1] = gy_at(r, y0 - 4 + m);
        Xp[r] = 0.f;
        if (ok[r] && y0 > 0) {
            const long long i = ib[r] + (y0 - 1) * sy;
            Xp[r] = -segy[i] * S.w[2][i];
        }
    }
    for (int y = y0; y < y1; ++y) {
        const long long py = y * sy;
        float pt[R], gr[R], xz0[R], xz1[R], xx0[R], xx1[R], xy0[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int m = 0; m < 7; ++m) Gq[r][m] = Gq[r][m + 1];
            Gq[r][7] = gy_at(r, y + 3);
            const int gz = z0 + lzr[r], gx = x0 + lxr[r];
            const long long i = ib[r] + py;
            pt[r] = S.q[i];
            gr[r] = S.gr[i];
            xz0[r] = -segz[i] * S.w[0][i];
            xz1[r] = (ok[r] && gz > 0) ? -segz[i - 1] * S.w[0][i - 1] : 0.f;
            xx0[r] = -segx[i] * S.w[1][i];
            xx1[r] = (ok[r] && gx > 0) ? -segx[i - sx] * S.w[1][i - sx] : 0.f;
            xy0[r] = -segy[i] * S.w[2][i];
        }
        __syncthreads();
        auto lz_ = [&](int lz, int lx, int c) {
            const int gz = z0 + lz - HW, gx = x0 + lx - HW;
            float g = 0.f;
            if ((unsigned)gz < (unsigned)nz && (unsigned)gx < (unsigned)nx) {
                const long long i = gx * sx + gz + py;
                const float h = -S.bdt[0][i] * S.w[0][i];
                const float a = achz[gz];
                g = a != 0.f ? h + a * (S.xi[0][i] + h) : h;
            }
            sgz[c] = g;
        };
        auto lx_ = [&](int lz, int lx, int c) {
            const int gz = z0 + lz - HW, gx = x0 + lx - HW;
            float g = 0.f;
            if ((unsigned)gz < (unsigned)nz && (unsigned)gx < (unsigned)nx) {
                const long long i = gx * sx + gz + py;
                const float h = -S.bdt[1][i] * S.w[1][i];
                const float a = achx[gx];
                g = a != 0.f ? h + a * (S.xi[1][i] + h) : h;
            }
            sgx[c] = g;
        };
        region3<T::LZ>(0, T::LZ, HW, HW + BX, lz_);
        region3<T::LZ>(HW, HW + BZ, 0, T::LX, lx_);
        __syncthreads();
        const float ay = aciy[y];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!ok[r]) continue;
            const int gz = z0 + lzr[r], gx = x0 + lxr[r];
            const long long i = ib[r] + py;
            const int c = (lxr[r] + HW) * T::LZ + lzr[r] + HW;
            const float az = aciz[gz], ax = acix[gx];
            if (az != 0.f || ax != 0.f || ay != 0.f) {
                const float qt = -S.kdt[i] * pt[r];
                if (az != 0.f) S.eta[0][i] = bciz[gz] * (S.eta[0][i] + qt);
                if (ax != 0.f) S.eta[1][i] = bcix[gx] * (S.eta[1][i] + qt);
                if (ay != 0.f) S.eta[2][i] = bciy[y] * (S.eta[2][i] + qt);
            }
            S.gr[i] = gr[r] + ((0.5f * (xz0[r] + xz1[r]) + 0.5f * (xx0[r] + xx1[r])) + 0.5f * (xy0[r] + Xp[r]));
            Xp[r] = xy0[r];
            const float dz = d_node(sgz, c, 1, C.c[0]);
            const float dx = d_node(sgx, c, T::LZ, C.c[1]);
            const float dy = d_queue(Gq[r], C.c[2]);
            S.q[i] = pt[r] - ((dz + dx) + dy);
        }
    }
}

// ---------------------------------------------------------------------------
template <int BZ, int BX, int BY>
static hipError_t launch3_t(int kind, int ntiles, hipStream_t st, const Slot* slots,
                            const int4* tiles, const Coef& C, int n, int sstep, int flag)
{
    dim3 g(ntiles), b(NTHREADS);
    const DSlot* ds = dev_slots(slots);
    switch (kind) {
    case K_BG_V:    k3_v<BZ, BX, BY, false, false><<<g, b, 0, st>>>(ds, tiles, C, n, sstep, flag); break;
    case K_BG_P:    k3_p<BZ, BX, BY, false, false><<<g, b, 0, st>>>(ds, tiles, C, n, sstep, flag); break;
    case K_SEG_V:   k3_v<BZ, BX, BY, false, true><<<g, b, 0, st>>>(ds, tiles, C, n, sstep, flag); break;
    case K_SEG_P:   k3_p<BZ, BX, BY, false, true><<<g, b, 0, st>>>(ds, tiles, C, n, sstep, flag); break;
    case K_BORN_V:  k3_v<BZ, BX, BY, true, false><<<g, b, 0, st>>>(ds, tiles, C, n, sstep, flag); break;
    case K_BORN_P:  k3_p<BZ, BX, BY, true, false><<<g, b, 0, st>>>(ds, tiles, C, n, sstep, flag); break;
    case K_ADJ_A:   k3_a<BZ, BX, BY><<<g, b, 0, st>>>(ds, tiles, C, n, sstep, flag); break;
    case K_ADJ_B:   k3_b<BZ, BX, BY><<<g, b, 0, st>>>(ds, tiles, C, n, sstep, flag); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

const int kTiles3[][3] = {{64, 4, 32}, {64, 8, 32}, {64, 8, 64}, {32, 8, 64}, {128, 4, 64}, {64, 4, 64}};
const int kNumTiles3 = 6;

hipError_t launch3d(int kind, int tile_id, int ntiles, hipStream_t st, const Slot* slots,
                    const int4* tiles, const Coef& C, int n, int sstep, int flag)
{
    if (ntiles <= 0) return hipSuccess;
    switch (tile_id) {
    case 0: return launch3_t<64, 4, 32>(kind, ntiles, st, slots, tiles, C, n, sstep, flag);
    case 1: return launch3_t<64, 8, 32>(kind, ntiles, st, slots, tiles, C, n, sstep, flag);
    case 2: return launch3_t<64, 8, 64>(kind, ntiles, st, slots, tiles, C, n, sstep, flag);
    case 3: return launch3_t<32, 8, 64>(kind, ntiles, st, slots, tiles, C, n, sstep, flag);
    case 4: return launch3_t<128, 4, 64>(kind, ntiles, st, slots, tiles, C, n, sstep, flag);
    case 5: return launch3_t<64, 4, 64>(kind, ntiles, st, slots, tiles, C, n, sstep, flag);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace lsrtm
