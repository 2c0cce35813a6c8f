// 2D stencil kernels of the velocity-pressure propagator (gfx950).
//
// Every launch advances all shots ("slots") of a launch group by one phase of
// one time step.  The grid walks a tile table: tile t = (slot, z0, x0) covers
// BZ x BX nodes of that slot's padded grid, R = BZ*BX/256 nodes per thread.
// The input of the phase's derivative is staged in LDS with the 4-node halo
// that derivative needs (z-halo for z-derivatives, x-halo for
// x-derivatives).  Each thread issues every global load it makes before the
// barrier at once -- the arrays it reads pointwise and its share of the
// staged cells, from addresses that are always valid (clamped to element 0
// where a cell lies outside the grid or a value is not needed), so that no
// branch separates them -- and only then combines the values and writes LDS.
// After one barrier every node is updated and written once, coalesced along
// z.  Values outside the padded grid are zero, as the discrete operators
// define them.
//
// Phases (section 2 of the paper, first-order system and eq. scattereqln;
// appendix A for the adjoint):
//   V : v_a <- v_a - dt b_a (G_a p + psi_a), with the CPML memory psi_a
//       advanced in the strips.  BORN adds the scattered velocity with the
//       density source -avg(dlnrho) dv_a; SEG stores G_a p + psi_a (the
//       gradient behind dv_a) for migration.
//   P : p <- p - dt kappa q, q = sum_a (D_a v_a + phi_a), plus the source.
//       BORN adds the scattered pressure with the bulk-modulus source
//       dlnkappa (-dt kappa q); SEG stores q for migration.
//   BORN and SEG together: the scattered V and P phases alone, the background
//       G_a p + psi_a and q of the step read from a replay buffer that a
//       migration pass filled (they are what the background phases would
//       compute, bit for bit); the background fields are not touched.
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
    static constexpr int R = NP / NTHREADS;
    static_assert(NP % NTHREADS == 0, "tile must hold a multiple of 256 nodes");
};

// Node r of this thread in the tile.
template <int BZ>
__device__ __forceinline__ void node_of(int r, int& lz, int& lx) {
    const int e = threadIdx.x + NTHREADS * r;
    lz = e % BZ;
    lx = e / BZ;
}

// Whether a tile (with the halo its staging reads) reaches a CPML strip; the
// tiles that do not (most of them) skip every CPML coefficient and memory
// load -- the coefficients are zero there.  Uniform over the workgroup.
template <int BZ, int BX>
__device__ __forceinline__ bool tile_in_pml(int z0, int x0, int nz, int nx, int npml) {
    return z0 - HW - 1 < npml || z0 + BZ + HW >= nz - npml - 1 ||
           x0 - HW - 1 < npml || x0 + BX + HW >= nx - npml - 1;
}

// ---------------------------------------------------------------------------
// V phase
// ---------------------------------------------------------------------------
template <int BZ, int BX, bool BORN, bool SEG>
__global__ void __launch_bounds__(NTHREADS)
k2_v(const DSlot* __restrict__ slots, const int4* __restrict__ tiles, Coef C, int n, int sstep, int flag, TileRec tr)
{
    using T = Tile2<BZ, BX>;
    constexpr int R = T::R;
    // BORN && SEG: the scattered phase alone on a background read from the
    // replay cache (the stored G_a p + psi_a of this step); the background
    // fields are neither read nor written
    constexpr bool CB = BORN && SEG;
    constexpr int K = BORN && !CB ? 2 : 1;
    using RZ = Cells<0, T::LZ, HW, BX>;                    // interior columns with the z-halo
    using RX = Cells<HW, BZ, 0, 2 * HW, 0, 0, HW, BX>;     // both x-halo strips
    __shared__ float sp[CB ? 1 : T::NL];
    __shared__ float sq[BORN ? T::NL : 1];
    const int tix = xcd_remap(blockIdx.x, gridDim.x);
    const int4 tl = tiles[tix];
    const DSlot& S = slots[tl.x];
    const int z0 = tl.y, x0 = tl.z;
    const int nz = S.n[0], nx = S.n[1];
    const unsigned ldz = (unsigned)S.ldz;
    const int npml = S.npml;
    const gfloat* achz = S.cpml[0];
    const gfloat* bchz = S.cpml[0] + nz;
    const gfloat* achx = S.cpml[1];
    const gfloat* bchx = S.cpml[1] + nx;
    const bool pml = tile_in_pml<BZ, BX>(z0, x0, nz, nx, npml);
    gfloat* __restrict__ seg = S.seg + (long long)sstep * 3 * S.npts;
    // pointwise loads, CPML coefficients and (inside the strips) memories
    float vz[R], vx[R], s0[R], s1z[R], s1x[R], wz[R], wx[R], r0[R], r1z[R], r1x[R];
    float az[R], ax[R], cz[R], cx[R], m0[R], m1[R], n0[R], n1[R];
    bool ok[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int lz, lx;
        node_of<BZ>(r, lz, lx);
        const int gz = z0 + lz, gx = x0 + lx;
        ok[r] = gz < nz && gx < nx;
        const unsigned i = ok[r] ? gx * ldz + gz : 0;
        const unsigned iz = ok[r] && in_pml(gz, nz, npml) ? i : 0;
        const unsigned ix = ok[r] && in_pml(gx, nx, npml) ? i : 0;
        vz[r] = CB ? elem(seg, i) : elem(S.v[0], i);            // cached: G_z p + psi_z
        vx[r] = CB ? elem(seg, S.npts + i) : elem(S.v[1], i);   // cached: G_x p + psi_x
        s0[r] = elem(S.sb, i);   // dt b_a = sb at the node times sb at its upper neighbour
        s1z[r] = elem(S.sb, gz + 1 < nz ? i + 1 : i);
        s1x[r] = elem(S.sb, gx + 1 < nx ? i + ldz : i);
        az[r] = pml ? elem(achz, ok[r] ? gz : 0) : 0.f;
        ax[r] = pml ? elem(achx, ok[r] ? gx : 0) : 0.f;
        cz[r] = pml ? elem(bchz, ok[r] ? gz : 0) : 0.f;
        cx[r] = pml ? elem(bchx, ok[r] ? gx : 0) : 0.f;
        m0[r] = pml && !CB ? elem(S.psi[0], iz) : 0.f;
        m1[r] = pml && !CB ? elem(S.psi[1], ix) : 0.f;
        if (BORN) {
            n0[r] = pml ? elem(S.xi[0], iz) : 0.f;
            n1[r] = pml ? elem(S.xi[1], ix) : 0.f;
            wz[r] = elem(S.w[0], i);
            wx[r] = elem(S.w[1], i);
            r0[r] = elem(S.dlnr, i);
            r1z[r] = elem(S.dlnr, gz + 1 < nz ? i + 1 : i);
            r1x[r] = elem(S.dlnr, gx + 1 < nx ? i + ldz : i);
        }
    }
    // stage p (and dp): cross of z- and x-halos
    auto inside = [&](int lz, int lx) {
        return (unsigned)(z0 + lz - HW) < (unsigned)nz && (unsigned)(x0 + lx - HW) < (unsigned)nx;
    };
    auto ld = [&](int lz, int lx, float* v) {
        const unsigned i = inside(lz, lx) ? (x0 + lx - HW) * ldz + (z0 + lz - HW) : 0;
        if (CB) {
            v[0] = elem(S.q, i);
        } else {
            v[0] = elem(S.p, i);
            if (BORN) v[1] = elem(S.q, i);
        }
    };
    auto st = [&](int lz, int lx, const float* v) {
        const int c = lx * T::LZ + lz;
        const bool in = inside(lz, lx);
        if (CB) {
            sq[c] = in ? v[0] : 0.f;
        } else {
            sp[c] = in ? v[0] : 0.f;
            if (BORN) sq[c] = in ? v[1] : 0.f;
        }
    };
    float hz[RZ::IT][K], hx[RX::IT][K];
    RZ::load(ld, hz);
    RX::load(ld, hx);
    RZ::store(st, hz);
    RX::store(st, hx);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!ok[r]) continue;
        int lz, lx;
        node_of<BZ>(r, lz, lx);
        const int gz = z0 + lz, gx = x0 + lx;
        const unsigned i = gx * ldz + gz;
        const int c = (lx + HW) * T::LZ + lz + HW;
        float gzp = vz[r], gxp = vx[r];
        if (!CB) {
            gzp = d_half(sp, c, 1, C.c[0]);
            gxp = d_half(sp, c, T::LZ, C.c[1]);
            if (az[r] != 0.f) {
                const float ps = fmaf(cz[r], m0[r], az[r] * gzp);
                elem(S.psi[0], i) = ps;
                gzp = gzp + ps;
            }
            if (ax[r] != 0.f) {
                const float ps = fmaf(cx[r], m1[r], ax[r] * gxp);
                elem(S.psi[1], i) = ps;
                gxp = gxp + ps;
            }
        }
        const float bz = s0[r] * s1z[r], bx = s0[r] * s1x[r];
        const float dvz = -bz * gzp;
        const float dvx = -bx * gxp;
        if (!CB) {
            elem(S.v[0], i) = vz[r] + dvz;
            elem(S.v[1], i) = vx[r] + dvx;
        }
        if (SEG && !BORN) {
            // the replay buffer is read back only k steps later: streaming stores
            __builtin_nontemporal_store(gzp, &elem(seg, i));
            __builtin_nontemporal_store(gxp, &elem(seg, S.npts + i));
        }
        if (!BORN && !SEG && (flag & PH_ACCUMULATE)) {   // pseudo-Hessian: sum of dv_a^2
            elem(S.w[0], i) = elem(S.w[0], i) + dvz * dvz;
            elem(S.w[1], i) = elem(S.w[1], i) + dvx * dvx;
        }
        if (BORN) {
            float gzq = d_half(sq, c, 1, C.c[0]);
            float gxq = d_half(sq, c, T::LZ, C.c[1]);
            if (az[r] != 0.f) {
                const float ps = fmaf(cz[r], n0[r], az[r] * gzq);
                elem(S.xi[0], i) = ps;
                gzq = gzq + ps;
            }
            if (ax[r] != 0.f) {
                const float ps = fmaf(cx[r], n1[r], ax[r] * gxq);
                elem(S.xi[1], i) = ps;
                gxq = gxq + ps;
            }
            const float rz = 0.5f * (r0[r] + r1z[r]);
            const float rx = 0.5f * (r0[r] + r1x[r]);
            elem(S.w[0], i) = (wz[r] - bz * gzq) - rz * dvz;
            elem(S.w[1], i) = (wx[r] - bx * gxq) - rx * dvx;
        }
    }
}

// ---------------------------------------------------------------------------
// P phase
// ---------------------------------------------------------------------------
template <int BZ, int BX, bool BORN, bool SEG>
__global__ void __launch_bounds__(NTHREADS)
k2_p(const DSlot* __restrict__ slots, const int4* __restrict__ tiles, Coef C, int n, int sstep, int flag, TileRec tr)
{
    using T = Tile2<BZ, BX>;
    constexpr int R = T::R;
    // BORN && SEG: the scattered phase alone, q of this step read from the
    // replay cache; the background fields are neither read nor written
    constexpr bool CB = BORN && SEG;
    constexpr int K = BORN && !CB ? 2 : 1;
    using RZ = Cells<0, T::LZ, HW, BX>;   // v_z (and w_z) with the z-halo
    using RX = Cells<HW, BZ, 0, T::LX>;   // v_x (and w_x) with the x-halo
    __shared__ float svz[CB ? 1 : T::NL];
    __shared__ float svx[CB ? 1 : T::NL];
    __shared__ float swz[BORN ? T::NL : 1];
    __shared__ float swx[BORN ? T::NL : 1];
    const int tix = xcd_remap(blockIdx.x, gridDim.x);
    const int4 tl = tiles[tix];
    const DSlot& S = slots[tl.x];
    const int z0 = tl.y, x0 = tl.z;
    const int nz = S.n[0], nx = S.n[1];
    const unsigned ldz = (unsigned)S.ldz;
    const int npml = S.npml;
    const gfloat* aciz = S.cpml[0] + 2 * nz;
    const gfloat* bciz = S.cpml[0] + 3 * nz;
    const gfloat* acix = S.cpml[1] + 2 * nx;
    const gfloat* bcix = S.cpml[1] + 3 * nx;
    const bool pml = tile_in_pml<BZ, BX>(z0, x0, nz, nx, npml);
    gfloat* __restrict__ seg = S.seg + (long long)sstep * 3 * S.npts + 2 * S.npts;
    // pointwise loads, CPML coefficients and (inside the strips) memories
    float pp[R], kk[R], qq[R], lk[R], az[R], ax[R], cz[R], cx[R], m0[R], m1[R], n0[R], n1[R];
    bool ok[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int lz, lx;
        node_of<BZ>(r, lz, lx);
        const int gz = z0 + lz, gx = x0 + lx;
        ok[r] = gz < nz && gx < nx;
        const unsigned i = ok[r] ? gx * ldz + gz : 0;
        const unsigned iz = ok[r] && in_pml(gz, nz, npml) ? i : 0;
        const unsigned ix = ok[r] && in_pml(gx, nx, npml) ? i : 0;
        pp[r] = CB ? elem(seg, i) : elem(S.p, i);   // cached: q
        kk[r] = elem(S.kdt, i);
        az[r] = pml ? elem(aciz, ok[r] ? gz : 0) : 0.f;
        ax[r] = pml ? elem(acix, ok[r] ? gx : 0) : 0.f;
        cz[r] = pml ? elem(bciz, ok[r] ? gz : 0) : 0.f;
        cx[r] = pml ? elem(bcix, ok[r] ? gx : 0) : 0.f;
        m0[r] = pml && !CB ? elem(S.phi[0], iz) : 0.f;
        m1[r] = pml && !CB ? elem(S.phi[1], ix) : 0.f;
        if (BORN) {
            qq[r] = elem(S.q, i);
            lk[r] = elem(S.dlnk, i);
            n0[r] = pml ? elem(S.eta[0], iz) : 0.f;
            n1[r] = pml ? elem(S.eta[1], ix) : 0.f;
        }
    }
    auto inside = [&](int lz, int lx) {
        return (unsigned)(z0 + lz - HW) < (unsigned)nz && (unsigned)(x0 + lx - HW) < (unsigned)nx;
    };
    auto index = [&](int lz, int lx) -> unsigned {
        return inside(lz, lx) ? (x0 + lx - HW) * ldz + (z0 + lz - HW) : 0;
    };
    auto ldz_ = [&](int lz, int lx, float* v) {
        const unsigned i = index(lz, lx);
        if (CB) {
            v[0] = elem(S.w[0], i);
        } else {
            v[0] = elem(S.v[0], i);
            if (BORN) v[1] = elem(S.w[0], i);
        }
    };
    auto ldx_ = [&](int lz, int lx, float* v) {
        const unsigned i = index(lz, lx);
        if (CB) {
            v[0] = elem(S.w[1], i);
        } else {
            v[0] = elem(S.v[1], i);
            if (BORN) v[1] = elem(S.w[1], i);
        }
    };
    auto stz_ = [&](int lz, int lx, const float* v) {
        const int c = lx * T::LZ + lz;
        const bool in = inside(lz, lx);
        if (CB) {
            swz[c] = in ? v[0] : 0.f;
        } else {
            svz[c] = in ? v[0] : 0.f;
            if (BORN) swz[c] = in ? v[1] : 0.f;
        }
    };
    auto stx_ = [&](int lz, int lx, const float* v) {
        const int c = lx * T::LZ + lz;
        const bool in = inside(lz, lx);
        if (CB) {
            swx[c] = in ? v[0] : 0.f;
        } else {
            svx[c] = in ? v[0] : 0.f;
            if (BORN) swx[c] = in ? v[1] : 0.f;
        }
    };
    float hz[RZ::IT][K], hx[RX::IT][K];
    RZ::load(ldz_, hz);
    RX::load(ldx_, hx);
    RZ::store(stz_, hz);
    RX::store(stx_, hx);
    const float amp = S.src >= 0 ? elem(S.src_amp, n) : 0.f;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!ok[r]) continue;
        int lz, lx;
        node_of<BZ>(r, lz, lx);
        const int gz = z0 + lz, gx = x0 + lx;
        const unsigned i = gx * ldz + gz;
        const int c = (lx + HW) * T::LZ + lz + HW;
        float q = pp[r];
        const float k = kk[r];
        if (!CB) {
            float ez = d_node(svz, c, 1, C.c[0]);
            float ex = d_node(svx, c, T::LZ, C.c[1]);
            if (az[r] != 0.f) {
                const float ph = fmaf(cz[r], m0[r], az[r] * ez);
                elem(S.phi[0], i) = ph;
                ez = ez + ph;
            }
            if (ax[r] != 0.f) {
                const float ph = fmaf(cx[r], m1[r], ax[r] * ex);
                elem(S.phi[1], i) = ph;
                ex = ex + ph;
            }
            q = ez + ex;
            float pn = pp[r] - k * q;
            if (i == S.src) pn = pn + amp;
            elem(S.p, i) = pn;
            if (SEG) __builtin_nontemporal_store(q, &elem(seg, i));
            if (!BORN && !SEG && (flag & PH_ACCUMULATE)) elem(S.gk, i) = elem(S.gk, i) + q * q;   // pseudo-Hessian: sum of q^2
            if (!BORN && tr.d) tile_gather(tr, tix, lz + BZ * lx, n, pn);
        }
        if (BORN) {
            float fz = d_node(swz, c, 1, C.c[0]);
            float fx = d_node(swx, c, T::LZ, C.c[1]);
            if (az[r] != 0.f) {
                const float ph = fmaf(cz[r], n0[r], az[r] * fz);
                elem(S.eta[0], i) = ph;
                fz = fz + ph;
            }
            if (ax[r] != 0.f) {
                const float ph = fmaf(cx[r], n1[r], ax[r] * fx);
                elem(S.eta[1], i) = ph;
                fx = fx + ph;
            }
            const float dq = fz + fx;
            const float qn = (qq[r] - k * dq) + lk[r] * (-k * q);
            elem(S.q, i) = qn;
            if (tr.d) tile_gather(tr, tix, lz + BZ * lx, n, qn);
        }
    }
}

// ---------------------------------------------------------------------------
// The adjoint state is kept scaled: Q = q~ = -dt kappa p~ in place of p~ and
// U_a = -dt b_a v~_a in place of v~_a (the same fields, one FP32 rounding
// apart), so that neither adjoint phase reads dt kappa or dt b_a at halo
// cells.  The replay buffer holds the CPML-corrected gradient G_a p + psi_a,
// so the lnrho image product -dv_a v~_a is -(G_a p + psi_a) U_a.
//
// Adjoint phase A (transpose of P): g_kappa += q^n Q;
// e~_a = Q + aci_a (phi~_a + Q);  v~_a -= G_a e~_a, i.e. U_a += dt b_a G_a e~_a;
// the pending chi update uses U_a before that.
// flag = 1 on the first reverse step (no pending chi update).
// ---------------------------------------------------------------------------
template <int BZ, int BX>
__global__ void __launch_bounds__(NTHREADS)
k2_a(const DSlot* __restrict__ slots, const int4* __restrict__ tiles, Coef C, int n, int sstep, int flag, TileRec tr)
{
    using T = Tile2<BZ, BX>;
    constexpr int R = T::R;
    using RZ = Cells<0, 2 * HW, HW, BX, HW, BZ>;          // both z-halo strips
    using RX = Cells<HW, BZ, 0, 2 * HW, 0, 0, HW, BX>;    // both x-halo strips
    __shared__ float sez[T::NL];
    __shared__ float sex[T::NL];
    const int tix = xcd_remap(blockIdx.x, gridDim.x);
    const int4 tl = tiles[tix];
    const DSlot& S = slots[tl.x];
    const int z0 = tl.y, x0 = tl.z;
    const int nz = S.n[0], nx = S.n[1], npml = S.npml;
    const unsigned ldz = (unsigned)S.ldz;
    const gfloat* __restrict__ segq = S.seg + (long long)sstep * 3 * S.npts + 2 * S.npts;
    const gfloat* aciz = S.cpml[0] + 2 * nz;
    const gfloat* acix = S.cpml[1] + 2 * nx;
    const bool pml = tile_in_pml<BZ, BX>(z0, x0, nz, nx, npml);
    auto inside = [&](int lz, int lx) {
        return (unsigned)(z0 + lz - HW) < (unsigned)nz && (unsigned)(x0 + lx - HW) < (unsigned)nx;
    };
    // loads of e~ at a cell: Q, then per wanted axis the CPML coefficient and
    // phi~ (the latter only inside the strips)
    auto lde = [&](int lz, int lx, float* v, bool wz, bool wx) {
        const int gz = z0 + lz - HW, gx = x0 + lx - HW;
        const bool in = inside(lz, lx);
        const unsigned i = in ? gx * ldz + gz : 0;
        v[0] = elem(S.q, i);
        if (wz) {
            v[1] = pml ? elem(aciz, in ? gz : 0) : 0.f;
            v[2] = pml ? elem(S.eta[0], in && in_pml(gz, nz, npml) ? i : 0) : 0.f;
        }
        if (wx) {
            v[3] = pml ? elem(acix, in ? gx : 0) : 0.f;
            v[4] = pml ? elem(S.eta[1], in && in_pml(gx, nx, npml) ? i : 0) : 0.f;
        }
    };
    auto ete = [&](bool in, const float* v, bool wz, bool wx, float& ez, float& ex, float& qt) {
        ez = ex = qt = 0.f;
        if (in) {
            qt = v[0];
            ez = qt;
            ex = qt;
            if (wz && v[1] != 0.f) ez = qt + v[1] * (v[2] + qt);
            if (wx && v[3] != 0.f) ex = qt + v[3] * (v[4] + qt);
        }
    };
    const gfloat* achz = S.cpml[0];
    const gfloat* bchz = S.cpml[0] + nz;
    const gfloat* achx = S.cpml[1];
    const gfloat* bchx = S.cpml[1] + nx;
    // the tile's own nodes need both components; Q is kept for the image and
    // sb at the node and its upper neighbours for dt b_a.  Unless this is the
    // first reverse step, the pending chi update needs the CPML coefficients
    // and chi at the node (inside the strips).
    float vz[R], vx[R], gk[R], qn[R], ev[R][5], s0[R], s1z[R], s1x[R];
    float hz_[R], hx_[R], cz[R], cx[R], xz[R], xx[R];
    bool ok[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int lz, lx;
        node_of<BZ>(r, lz, lx);
        const int gz = z0 + lz, gx = x0 + lx;
        ok[r] = gz < nz && gx < nx;
        const unsigned i = ok[r] ? gx * ldz + gz : 0;
        vz[r] = elem(S.w[0], i);
        vx[r] = elem(S.w[1], i);
        gk[r] = __builtin_nontemporal_load(&elem(S.gk, i));   // read once: leaves L2 / the
                                                              // Infinity Cache to the adjoint state
        qn[r] = __builtin_nontemporal_load(&elem(segq, i));
        s0[r] = elem(S.sb, i);
        s1z[r] = elem(S.sb, gz + 1 < nz ? i + 1 : i);
        s1x[r] = elem(S.sb, gx + 1 < nx ? i + ldz : i);
        lde(lz + HW, lx + HW, ev[r], true, true);
        if (!flag && pml) {
            const unsigned iz = ok[r] && in_pml(gz, nz, npml) ? i : 0;
            const unsigned ix = ok[r] && in_pml(gx, nx, npml) ? i : 0;
            hz_[r] = elem(achz, ok[r] ? gz : 0);
            hx_[r] = elem(achx, ok[r] ? gx : 0);
            cz[r] = elem(bchz, ok[r] ? gz : 0);
            cx[r] = elem(bchx, ok[r] ? gx : 0);
            xz[r] = elem(S.xi[0], iz);
            xx[r] = elem(S.xi[1], ix);
        } else {
            hz_[r] = hx_[r] = cz[r] = cx[r] = xz[r] = xx[r] = 0.f;
        }
    }
    float hz[RZ::IT][5], hx[RX::IT][5];
    RZ::load([&](int lz, int lx, float* v) { lde(lz, lx, v, true, false); }, hz);
    RX::load([&](int lz, int lx, float* v) { lde(lz, lx, v, false, true); }, hx);
    float qt[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int lz, lx;
        node_of<BZ>(r, lz, lx);
        float ez, ex;
        ete(ok[r], ev[r], true, true, ez, ex, qt[r]);
        const int c = (lx + HW) * T::LZ + lz + HW;
        sez[c] = ez;
        sex[c] = ex;
    }
    RZ::store([&](int lz, int lx, const float* v) {
        const int c = lx * T::LZ + lz;
        float ez, ex, q;
        ete(inside(lz, lx), v, true, false, ez, ex, q);
        sez[c] = ez;
    }, hz);
    RX::store([&](int lz, int lx, const float* v) {
        const int c = lx * T::LZ + lz;
        float ez, ex, q;
        ete(inside(lz, lx), v, false, true, ez, ex, q);
        sex[c] = ex;
    }, hx);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!ok[r]) continue;
        int lz, lx;
        node_of<BZ>(r, lz, lx);
        const int gz = z0 + lz, gx = x0 + lx;
        const unsigned i = gx * ldz + gz;
        const int c = (lx + HW) * T::LZ + lz + HW;
        if (!flag) {
            if (hz_[r] != 0.f) elem(S.xi[0], i) = cz[r] * (xz[r] + vz[r]);
            if (hx_[r] != 0.f) elem(S.xi[1], i) = cx[r] * (xx[r] + vx[r]);
        }
        __builtin_nontemporal_store(gk[r] + qn[r] * qt[r], &elem(S.gk, i));
        const float bz = s0[r] * s1z[r], bx = s0[r] * s1x[r];
        elem(S.w[0], i) = vz[r] + bz * d_half(sez, c, 1, C.c[0]);
        elem(S.w[1], i) = vx[r] + bx * d_half(sex, c, T::LZ, C.c[1]);
    }
}

// ---------------------------------------------------------------------------
// Adjoint phase B (transpose of V): phi~_a <- bci_a (phi~_a + Q);
// g_rho += avg^T(-dv_a v~_a) = avg^T(-(G_a p + psi_a) U_a);  h~_a = U_a,
// g~_a = h~_a + ach_a (chi_a + h~_a);  p~ -= sum_a D_a g~_a (and the adjoint
// source is added to p~), i.e. Q += dt kappa (sum_a D_a g~_a - source).
// The image products are formed while staging (the transpose of the
// half-node average needs them at the node and at its lower neighbour).
// ---------------------------------------------------------------------------
template <int BZ, int BX>
__global__ void __launch_bounds__(NTHREADS)
k2_b(const DSlot* __restrict__ slots, const int4* __restrict__ tiles, Coef C, int n, int sstep, int flag, TileRec tr)
{
    using T = Tile2<BZ, BX>;
    constexpr int R = T::R;
    using RZ = Cells<0, T::LZ, HW, BX>;   // g~_z with the z-halo
    using RX = Cells<HW, BZ, 0, T::LX>;   // g~_x with the x-halo
    __shared__ float sgz[T::NL];
    __shared__ float sgx[T::NL];
    __shared__ float sxz[T::NL];
    __shared__ float sxx[T::NL];
    const int tix = xcd_remap(blockIdx.x, gridDim.x);
    const int4 tl = tiles[tix];
    const DSlot& S = slots[tl.x];
    const int z0 = tl.y, x0 = tl.z;
    const int nz = S.n[0], nx = S.n[1], npml = S.npml;
    const unsigned ldz = (unsigned)S.ldz;
    const gfloat* __restrict__ segz = S.seg + (long long)sstep * 3 * S.npts;
    const gfloat* __restrict__ segx = segz + S.npts;
    const gfloat* aciz = S.cpml[0] + 2 * nz;
    const gfloat* bciz = S.cpml[0] + 3 * nz;
    const gfloat* acix = S.cpml[1] + 2 * nx;
    const gfloat* bcix = S.cpml[1] + 3 * nx;
    const bool pml = tile_in_pml<BZ, BX>(z0, x0, nz, nx, npml);
    // pointwise loads: Q, g_rho and dt kappa; the phi~ update needs the CPML
    // coefficients and phi~ at the node (inside the strips)
    float pt[R], gr[R], az[R], ax[R], cz[R], cx[R], ez[R], ex[R], kk[R];
    bool ok[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int lz, lx;
        node_of<BZ>(r, lz, lx);
        const int gz = z0 + lz, gx = x0 + lx;
        ok[r] = gz < nz && gx < nx;
        const unsigned i = ok[r] ? gx * ldz + gz : 0;
        const bool mz = ok[r] && in_pml(gz, nz, npml), mx = ok[r] && in_pml(gx, nx, npml);
        pt[r] = elem(S.q, i);
        gr[r] = elem(S.gr, i);
        az[r] = pml ? elem(aciz, ok[r] ? gz : 0) : 0.f;
        ax[r] = pml ? elem(acix, ok[r] ? gx : 0) : 0.f;
        cz[r] = pml ? elem(bciz, ok[r] ? gz : 0) : 0.f;
        cx[r] = pml ? elem(bcix, ok[r] ? gx : 0) : 0.f;
        ez[r] = pml ? elem(S.eta[0], mz ? i : 0) : 0.f;
        ex[r] = pml ? elem(S.eta[1], mx ? i : 0) : 0.f;
        kk[r] = elem(S.kdt, i);
    }
    const gfloat* achz = S.cpml[0];
    const gfloat* achx = S.cpml[1];
    auto inside = [&](int lz, int lx) {
        return (unsigned)(z0 + lz - HW) < (unsigned)nz && (unsigned)(x0 + lx - HW) < (unsigned)nx;
    };
    // loads of g~_a and of the image product at a cell: the CPML coefficient,
    // chi_a (inside the strips only), U_a and G_a p + psi_a (on the rows or
    // columns whose product is needed).  This order keeps the compiler's
    // schedule of the staging loads in one batch (54 VGPRs; other orders
    // split it into dependent groups at 66-67 VGPRs).
    auto ldz_ = [&](int lz, int lx, float* v) {
        const int gz = z0 + lz - HW, gx = x0 + lx - HW;
        const bool in = inside(lz, lx);
        const unsigned i = in ? gx * ldz + gz : 0;
        v[0] = pml ? elem(achz, in ? gz : 0) : 0.f;
        v[1] = pml ? elem(S.xi[0], in && in_pml(gz, nz, npml) ? i : 0) : 0.f;
        v[2] = elem(S.w[0], i);
        v[3] = elem(segz, in && lz >= HW - 1 && lz < HW + BZ ? i : 0);
    };
    auto ldx_ = [&](int lz, int lx, float* v) {
        const int gz = z0 + lz - HW, gx = x0 + lx - HW;
        const bool in = inside(lz, lx);
        const unsigned i = in ? gx * ldz + gz : 0;
        v[0] = pml ? elem(achx, in ? gx : 0) : 0.f;
        v[1] = pml ? elem(S.xi[1], in && in_pml(gx, nx, npml) ? i : 0) : 0.f;
        v[2] = elem(S.w[1], i);
        v[3] = elem(segx, in && lx >= HW - 1 && lx < HW + BX ? i : 0);
    };
    auto stz_ = [&](int lz, int lx, const float* v) {
        const int c = lx * T::LZ + lz;
        float g = 0.f, x = 0.f;
        if (inside(lz, lx)) {
            const float h = v[2];
            g = v[0] != 0.f ? h + v[0] * (v[1] + h) : h;
            if (lz >= HW - 1 && lz < HW + BZ) x = -v[3] * v[2];
        }
        sgz[c] = g;
        sxz[c] = x;
    };
    auto stx_ = [&](int lz, int lx, const float* v) {
        const int c = lx * T::LZ + lz;
        float g = 0.f, x = 0.f;
        if (inside(lz, lx)) {
            const float h = v[2];
            g = v[0] != 0.f ? h + v[0] * (v[1] + h) : h;
            if (lx >= HW - 1 && lx < HW + BX) x = -v[3] * v[2];
        }
        sgx[c] = g;
        sxx[c] = x;
    };
    float hz[RZ::IT][4], hx[RX::IT][4];
    RZ::load(ldz_, hz);
    RX::load(ldx_, hx);
    RZ::store(stz_, hz);
    RX::store(stx_, hx);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!ok[r]) continue;
        int lz, lx;
        node_of<BZ>(r, lz, lx);
        const int gz = z0 + lz, gx = x0 + lx;
        const unsigned i = gx * ldz + gz;
        const int c = (lx + HW) * T::LZ + lz + HW;
        if (az[r] != 0.f) elem(S.eta[0], i) = cz[r] * (ez[r] + pt[r]);
        if (ax[r] != 0.f) elem(S.eta[1], i) = cx[r] * (ex[r] + pt[r]);
        // transpose of the half-node average: the last node of an axis also
        // takes the other half of its own product (the forward average there
        // clamps the upper neighbour to the node itself)
        const float tz = 0.5f * (sxz[c] + sxz[c - 1]) + (gz + 1 == nz ? 0.5f * sxz[c] : 0.f);
        const float tx = 0.5f * (sxx[c] + sxx[c - T::LZ]) + (gx + 1 == nx ? 0.5f * sxx[c] : 0.f);
        elem(S.gr, i) = gr[r] + (tz + tx);
        const float dz = d_node(sgz, c, 1, C.c[0]);
        const float dx = d_node(sgx, c, T::LZ, C.c[1]);
        float qn = pt[r] + kk[r] * (dz + dx);
        if (tr.y && n > 0) qn = qn - kk[r] * tile_inject(tr, tix, lz + BZ * lx, n - 1);
        elem(S.q, i) = qn;
    }
}

// ---------------------------------------------------------------------------
// Host-side dispatch over tile shapes
// ---------------------------------------------------------------------------
template <int BZ, int BX>
static hipError_t launch2_t(int kind, int ntiles, hipStream_t st, const Slot* slots,
                            const int4* tiles, const Coef& C, int n, int sstep, int flag, const TileRec& tr,
                            hipEvent_t e0, hipEvent_t e1)
{
    dim3 g(ntiles), b(NTHREADS);
    const DSlot* ds = dev_slots(slots);
    switch (kind) {
    case K_BG_V:    launch_k(k2_v<BZ, BX, false, false>, g, b, st, e0, e1, ds, tiles, C, n, sstep, flag, tr); break;
    case K_BG_P:    launch_k(k2_p<BZ, BX, false, false>, g, b, st, e0, e1, ds, tiles, C, n, sstep, flag, tr); break;
    case K_SEG_V:   launch_k(k2_v<BZ, BX, false, true>, g, b, st, e0, e1, ds, tiles, C, n, sstep, flag, tr); break;
    case K_SEG_P:   launch_k(k2_p<BZ, BX, false, true>, g, b, st, e0, e1, ds, tiles, C, n, sstep, flag, tr); break;
    case K_BORN_V:  launch_k(k2_v<BZ, BX, true, false>, g, b, st, e0, e1, ds, tiles, C, n, sstep, flag, tr); break;
    case K_BORN_P:  launch_k(k2_p<BZ, BX, true, false>, g, b, st, e0, e1, ds, tiles, C, n, sstep, flag, tr); break;
    case K_BORN_V_RC: launch_k(k2_v<BZ, BX, true, true>, g, b, st, e0, e1, ds, tiles, C, n, sstep, flag, tr); break;
    case K_BORN_P_RC: launch_k(k2_p<BZ, BX, true, true>, g, b, st, e0, e1, ds, tiles, C, n, sstep, flag, tr); break;
    case K_ADJ_A:   launch_k(k2_a<BZ, BX>, g, b, st, e0, e1, ds, tiles, C, n, sstep, flag, tr); break;
    case K_ADJ_B:   launch_k(k2_b<BZ, BX>, g, b, st, e0, e1, ds, tiles, C, n, sstep, flag, tr); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

const int kTiles2[][2] = {{32, 8}, {32, 16}, {32, 32}, {64, 4}, {64, 8}, {64, 16},
                          {128, 4}, {128, 8}, {256, 4}};
const int kNumTiles2 = 9;

hipError_t launch2d(int kind, int tile_id, int ntiles, hipStream_t st, const Slot* slots,
                    const int4* tiles, const Coef& C, int n, int sstep, int flag, const TileRec& tr,
                            hipEvent_t e0, hipEvent_t e1)
{
    if (ntiles <= 0) return hipSuccess;
    switch (tile_id) {
    case 0: return launch2_t<32, 8>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, tr, e0, e1);
    case 1: return launch2_t<32, 16>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, tr, e0, e1);
    case 2: return launch2_t<32, 32>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, tr, e0, e1);
    case 3: return launch2_t<64, 4>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, tr, e0, e1);
    case 4: return launch2_t<64, 8>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, tr, e0, e1);
    case 5: return launch2_t<64, 16>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, tr, e0, e1);
    case 6: return launch2_t<128, 4>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, tr, e0, e1);
    case 7: return launch2_t<128, 8>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, tr, e0, e1);
    case 8: return launch2_t<256, 4>(kind, ntiles, st, slots, tiles, C, n, sstep, flag, tr, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace lsrtm
