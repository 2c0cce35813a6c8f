// 2D stencil kernels of the velocity-pressure propagator (gfx950).
//
// Every launch advances all shots ("slots") of a launch group by one phase of
// one time step.  The grid walks a tile table: tile t = (slot, z0, x0) covers
// BZ x BX nodes of that slot's padded grid.  The input field of the phase's
// derivative is staged with a 4-node halo in LDS; every other array is read
// and written once, coalesced along z.  Values outside the padded grid are
// zero, as the discrete operators define them.
//
// Phases (section 2 of the paper, first-order system and eq. scattereqln;
// appendix A for the adjoint):
//   V : v_a <- v_a - dt b_a (G_a p + psi_a), with the CPML memory psi_a
//       advanced in the strips.  BORN adds the scattered velocity with the
//       density source -avg(dlnrho) dv_a; SEG stores dv_a for migration.
//   P : p <- p - dt kappa q, q = sum_a (D_a v_a + phi_a), plus the source.
//       BORN adds the scattered pressure with the bulk-modulus source
//       dlnkappa (-dt kappa q); SEG stores q for migration.
//   A : adjoint pressure phase (transpose of P), imaging of lnkappa.
//   B : adjoint velocity phase (transpose of V), imaging of lnrho.
// The adjoint CPML memories are advanced in the phase that does not read them
// at halo nodes (phi~ in B, chi in the next step's A), so no tile overwrites
// a value another tile still needs.
#include "common.h"
#include "kernels.h"

namespace lsrtm {

template <int BZ, int BX>
struct Tile2 {
    static constexpr int LZ = BZ + 2 * HW;
    static constexpr int LX = BX + 2 * HW;
    static constexpr int NL = LZ * LX;
    static constexpr int NP = BZ * BX;
};

// ---------------------------------------------------------------------------
// V phase
// ---------------------------------------------------------------------------
template <int BZ, int BX, bool BORN, bool SEG>
__global__ void __launch_bounds__(NTHREADS)
k2_v(const Slot* __restrict__ slots, const int4* __restrict__ tiles, Coef C, int n, int sstep, int flag)
{
    using T = Tile2<BZ, BX>;
    __shared__ float sp[T::NL];
    __shared__ float sq[BORN ? T::NL : 1];
    const int4 tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const Slot& S = slots[tl.x];
    const int z0 = tl.y, x0 = tl.z;
    const int nz = S.n[0], nx = S.n[1];
    const long long ldz = S.ldz;
    const float* __restrict__ P = S.p;
    const float* __restrict__ Q = S.q;
    for (int e = threadIdx.x; e < T::NL; e += NTHREADS) {
        const int lz = e % T::LZ, lx = e / T::LZ;
        const int gz = z0 + lz - HW, gx = x0 + lx - HW;
        const bool in = (unsigned)gz < (unsigned)nz && (unsigned)gx < (unsigned)nx;
        const long long i = gx * ldz + gz;
        sp[e] = in ? P[i] : 0.f;
        if (BORN) sq[e] = in ? Q[i] : 0.f;
    }
    __syncthreads();
    const float* achz = S.cpml[0];
    const float* bchz = S.cpml[0] + nz;
    const float* achx = S.cpml[1];
    const float* bchx = S.cpml[1] + nx;
    float* __restrict__ seg = S.seg + (long long)sstep * 3 * S.npts;
    for (int e = threadIdx.x; e < T::NP; e += NTHREADS) {
        const int lz = e % BZ, lx = e / BZ;
        const int gz = z0 + lz, gx = x0 + lx;
        if (gz >= nz || gx >= nx) continue;
        const long long i = gx * ldz + gz;
        const int c = (lx + HW) * T::LZ + lz + HW;
        const float az = achz[gz], ax = achx[gx];
        const float bz = S.bdt[0][i], bx = S.bdt[1][i];
        // background
        float gzp = d_half(sp, c, 1, C.c[0]);
        float gxp = d_half(sp, c, T::LZ, C.c[1]);
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
        const float dvz = -bz * gzp;
        const float dvx = -bx * gxp;
        S.v[0][i] = S.v[0][i] + dvz;
        S.v[1][i] = S.v[1][i] + dvx;
        if (SEG) {
            seg[i] = dvz;
            seg[S.npts + i] = dvx;
        }
        if (BORN) {
            float gzq = d_half(sq, c, 1, C.c[0]);
            float gxq = d_half(sq, c, T::LZ, C.c[1]);
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
            const float r0 = S.dlnr[i];
            const float rz = 0.5f * (r0 + S.dlnr[gz + 1 < nz ? i + 1 : i]);
            const float rx = 0.5f * (r0 + S.dlnr[gx + 1 < nx ? i + ldz : i]);
            S.w[0][i] = (S.w[0][i] - bz * gzq) - rz * dvz;
            S.w[1][i] = (S.w[1][i] - bx * gxq) - rx * dvx;
        }
    }
}

// ---------------------------------------------------------------------------
// P phase
// ---------------------------------------------------------------------------
template <int BZ, int BX, bool BORN, bool SEG>
__global__ void __launch_bounds__(NTHREADS)
k2_p(const Slot* __restrict__ slots, const int4* __restrict__ tiles, Coef C, int n, int sstep, int flag)
{
    using T = Tile2<BZ, BX>;
    __shared__ float svz[T::NL];
    __shared__ float svx[T::NL];
    __shared__ float swz[BORN ? T::NL : 1];
    __shared__ float swx[BORN ? T::NL : 1];
    const int4 tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const Slot& S = slots[tl.x];
    const int z0 = tl.y, x0 = tl.z;
    const int nz = S.n[0], nx = S.n[1];
    const long long ldz = S.ldz;
    for (int e = threadIdx.x; e < T::NL; e += NTHREADS) {
        const int lz = e % T::LZ, lx = e / T::LZ;
        const int gz = z0 + lz - HW, gx = x0 + lx - HW;
        const bool in = (unsigned)gz < (unsigned)nz && (unsigned)gx < (unsigned)nx;
        const long long i = gx * ldz + gz;
        svz[e] = in ? S.v[0][i] : 0.f;
        svx[e] = in ? S.v[1][i] : 0.f;
        if (BORN) {
            swz[e] = in ? S.w[0][i] : 0.f;
            swx[e] = in ? S.w[1][i] : 0.f;
        }
    }
    __syncthreads();
    const float* aciz = S.cpml[0] + 2 * nz;
    const float* bciz = S.cpml[0] + 3 * nz;
    const float* acix = S.cpml[1] + 2 * nx;
    const float* bcix = S.cpml[1] + 3 * nx;
    const float amp = S.src >= 0 ? S.src_amp[n] : 0.f;
    float* __restrict__ seg = S.seg + (long long)sstep * 3 * S.npts + 2 * S.npts;
    for (int e = threadIdx.x; e < T::NP; e += NTHREADS) {
        const int lz = e % BZ, lx = e / BZ;
        const int gz = z0 + lz, gx = x0 + lx;
        if (gz >= nz || gx >= nx) continue;
        const long long i = gx * ldz + gz;
        const int c = (lx + HW) * T::LZ + lz + HW;
        const float az = aciz[gz], ax = acix[gx];
        float ez = d_node(svz, c, 1, C.c[0]);
        float ex = d_node(svx, c, T::LZ, C.c[1]);
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
        const float q = ez + ex;
        const float k = S.kdt[i];
        float pn = S.p[i] - k * q;
        if (i == S.src) pn = pn + amp;
        S.p[i] = pn;
        if (SEG) seg[i] = q;
        if (BORN) {
            float fz = d_node(swz, c, 1, C.c[0]);
            float fx = d_node(swx, c, T::LZ, C.c[1]);
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
            const float dq = fz + fx;
            S.q[i] = (S.q[i] - k * dq) + S.dlnk[i] * (-k * q);
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoint phase A (transpose of P): g_kappa += (-dt kappa q^n) p~;
// e~_a = q~ + aci_a (phi~_a + q~) with q~ = -dt kappa p~;  v~_a -= G_a e~_a.
// flag = 1 on the first reverse step (no pending chi update).
// ---------------------------------------------------------------------------
template <int BZ, int BX>
__global__ void __launch_bounds__(NTHREADS)
k2_a(const Slot* __restrict__ slots, const int4* __restrict__ tiles, Coef C, int n, int sstep, int flag)
{
    using T = Tile2<BZ, BX>;
    __shared__ float sez[T::NL];
    __shared__ float sex[T::NL];
    const int4 tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const Slot& S = slots[tl.x];
    const int z0 = tl.y, x0 = tl.z;
    const int nz = S.n[0], nx = S.n[1];
    const long long ldz = S.ldz;
    const float* aciz = S.cpml[0] + 2 * nz;
    const float* acix = S.cpml[1] + 2 * nx;
    for (int e = threadIdx.x; e < T::NL; e += NTHREADS) {
        const int lz = e % T::LZ, lx = e / T::LZ;
        const int gz = z0 + lz - HW, gx = x0 + lx - HW;
        const bool in = (unsigned)gz < (unsigned)nz && (unsigned)gx < (unsigned)nx;
        float ez = 0.f, ex = 0.f;
        if (in) {
            const long long i = gx * ldz + gz;
            const float qt = -S.kdt[i] * S.q[i];
            ez = qt;
            ex = qt;
            const float az = aciz[gz], ax = acix[gx];
            if (az != 0.f) ez = qt + az * (S.eta[0][i] + qt);
            if (ax != 0.f) ex = qt + ax * (S.eta[1][i] + qt);
        }
        sez[e] = ez;
        sex[e] = ex;
    }
    __syncthreads();
    const float* achz = S.cpml[0];
    const float* bchz = S.cpml[0] + nz;
    const float* achx = S.cpml[1];
    const float* bchx = S.cpml[1] + nx;
    const float* __restrict__ segq = S.seg + (long long)sstep * 3 * S.npts + 2 * S.npts;
    for (int e = threadIdx.x; e < T::NP; e += NTHREADS) {
        const int lz = e % BZ, lx = e / BZ;
        const int gz = z0 + lz, gx = x0 + lx;
        if (gz >= nz || gx >= nx) continue;
        const long long i = gx * ldz + gz;
        const int c = (lx + HW) * T::LZ + lz + HW;
        float vz = S.w[0][i], vx = S.w[1][i];
        if (!flag) {
            const float hz = achz[gz], hx = achx[gx];
            if (hz != 0.f) S.xi[0][i] = bchz[gz] * (S.xi[0][i] + (-S.bdt[0][i] * vz));
            if (hx != 0.f) S.xi[1][i] = bchx[gx] * (S.xi[1][i] + (-S.bdt[1][i] * vx));
        }
        const float k = S.kdt[i];
        S.gk[i] = S.gk[i] + (-k * segq[i]) * S.q[i];
        vz = vz - d_half(sez, c, 1, C.c[0]);
        vx = vx - d_half(sex, c, T::LZ, C.c[1]);
        S.w[0][i] = vz;
        S.w[1][i] = vx;
    }
}

// ---------------------------------------------------------------------------
// Adjoint phase B (transpose of V): phi~_a <- bci_a (phi~_a + q~);
// g_rho += avg^T(-dv_a v~_a);  h~_a = -dt b_a v~_a,
// g~_a = h~_a + ach_a (chi_a + h~_a);  p~ -= sum_a D_a g~_a.
// ---------------------------------------------------------------------------
template <int BZ, int BX>
__global__ void __launch_bounds__(NTHREADS)
k2_b(const Slot* __restrict__ slots, const int4* __restrict__ tiles, Coef C, int n, int sstep, int flag)
{
    using T = Tile2<BZ, BX>;
    __shared__ float sgz[T::NL];
    __shared__ float sgx[T::NL];
    const int4 tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const Slot& S = slots[tl.x];
    const int z0 = tl.y, x0 = tl.z;
    const int nz = S.n[0], nx = S.n[1];
    const long long ldz = S.ldz;
    const float* achz = S.cpml[0];
    const float* achx = S.cpml[1];
    for (int e = threadIdx.x; e < T::NL; e += NTHREADS) {
        const int lz = e % T::LZ, lx = e / T::LZ;
        const int gz = z0 + lz - HW, gx = x0 + lx - HW;
        const bool in = (unsigned)gz < (unsigned)nz && (unsigned)gx < (unsigned)nx;
        float gzv = 0.f, gxv = 0.f;
        if (in) {
            const long long i = gx * ldz + gz;
            const float hz = -S.bdt[0][i] * S.w[0][i];
            const float hx = -S.bdt[1][i] * S.w[1][i];
            gzv = hz;
            gxv = hx;
            const float az = achz[gz], ax = achx[gx];
            if (az != 0.f) gzv = hz + az * (S.xi[0][i] + hz);
            if (ax != 0.f) gxv = hx + ax * (S.xi[1][i] + hx);
        }
        sgz[e] = gzv;
        sgx[e] = gxv;
    }
    __syncthreads();
    const float* aciz = S.cpml[0] + 2 * nz;
    const float* bciz = S.cpml[0] + 3 * nz;
    const float* acix = S.cpml[1] + 2 * nx;
    const float* bcix = S.cpml[1] + 3 * nx;
    const float* __restrict__ segz = S.seg + (long long)sstep * 3 * S.npts;
    const float* __restrict__ segx = segz + S.npts;
    for (int e = threadIdx.x; e < T::NP; e += NTHREADS) {
        const int lz = e % BZ, lx = e / BZ;
        const int gz = z0 + lz, gx = x0 + lx;
        if (gz >= nz || gx >= nx) continue;
        const long long i = gx * ldz + gz;
        const int c = (lx + HW) * T::LZ + lz + HW;
        const float pt = S.q[i];
        const float qt = -S.kdt[i] * pt;
        const float az = aciz[gz], ax = acix[gx];
        if (az != 0.f) S.eta[0][i] = bciz[gz] * (S.eta[0][i] + qt);
        if (ax != 0.f) S.eta[1][i] = bcix[gx] * (S.eta[1][i] + qt);
        // lnrho imaging with the transpose of the half-node average
        const float xz0 = -segz[i] * S.w[0][i];
        const float xz1 = gz > 0 ? -segz[i - 1] * S.w[0][i - 1] : 0.f;
        const float xx0 = -segx[i] * S.w[1][i];
        const float xx1 = gx > 0 ? -segx[i - ldz] * S.w[1][i - ldz] : 0.f;
        S.gr[i] = S.gr[i] + (0.5f * (xz0 + xz1) + 0.5f * (xx0 + xx1));
        const float dz = d_node(sgz, c, 1, C.c[0]);
        const float dx = d_node(sgx, c, T::LZ, C.c[1]);
        S.q[i] = pt - (dz + dx);
    }
}

// ---------------------------------------------------------------------------
// Host-side dispatch over tile shapes
// ---------------------------------------------------------------------------
template <int BZ, int BX>
static hipError_t launch2_t(int kind, int ntiles, hipStream_t st, const Slot* slots,
                            const int4* tiles, const Coef& C, int n, int sstep, int flag)
{
    dim3 g(ntiles), b(NTHREADS);
    switch (kind) {
    case K_BG_V:    k2_v<BZ, BX, false, false><<<g, b, 0, st>>>(slots, tiles, C, n, sstep, flag); break;
    case K_BG_P:    k2_p<BZ, BX, false, false><<<g, b, 0, st>>>(slots, tiles, C, n, sstep, flag); break;
    case K_SEG_V:   k2_v<BZ, BX, false, true><<<g, b, 0, st>>>(slots, tiles, C, n, sstep, flag); break;
    case K_SEG_P:   k2_p<BZ, BX, false, true><<<g, b, 0, st>>>(slots, tiles, C, n, sstep, flag); break;
    case K_BORN_V:  k2_v<BZ, BX, true, false><<<g, b, 0, st>>>(slots, tiles, C, n, sstep, flag); break;
    case K_BORN_P:  k2_p<BZ, BX, true, false><<<g, b, 0, st>>>(slots, tiles, C, n, sstep, flag); break;
    case K_ADJ_A:   k2_a<BZ, BX><<<g, b, 0, st>>>(slots, tiles, C, n, sstep, flag); break;
    case K_ADJ_B:   k2_b<BZ, BX><<<g, b, 0, st>>>(slots, tiles, C, n, sstep, flag); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

const int kTiles2[][2] = {{32, 4}, {32, 8}, {32, 16}, {64, 4}, {64, 8}, {64, 16},
                          {128, 4}, {128, 8}, {128, 16}};
const int kNumTiles2 = 9;

hipError_t launch2d(int kind, int tile_id, int ntiles, hipStream_t st, const Slot* slots,
                    const int4* tiles, const Coef& C, int n, int sstep, int flag)
{
    if (ntiles <= 0) return hipSuccess;
    switch (tile_id) {
    case 0: return launch2_t<32, 4>(kind, ntiles, st, slots, tiles, C, n, sstep, flag);
    case 1: return launch2_t<32, 8>(kind, ntiles, st, slots, tiles, C, n, sstep, flag);
    case 2: return launch2_t<32, 16>(kind, ntiles, st, slots, tiles, C, n, sstep, flag);
    case 3: return launch2_t<64, 4>(kind, ntiles, st, slots, tiles, C, n, sstep, flag);
    case 4: return launch2_t<64, 8>(kind, ntiles, st, slots, tiles, C, n, sstep, flag);
    case 5: return launch2_t<64, 16>(kind, ntiles, st, slots, tiles, C, n, sstep, flag);
    case 6: return launch2_t<128, 4>(kind, ntiles, st, slots, tiles, C, n, sstep, flag);
    case 7: return launch2_t<128, 8>(kind, ntiles, st, slots, tiles, C, n, sstep, flag);
    case 8: return launch2_t<128, 16>(kind, ntiles, st, slots, tiles, C, n, sstep, flag);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace lsrtm
