// Interpolated point-spread-function Hessian (appendix C of the paper) for
// image-domain LSRTM (section 3, eq. migdeconobj).
//
// PSF images P[q][p] (response in parameter p to the scatterer lattice of
// parameter q, computed by one Born and one migration pass) sample columns of
// H = L^T L.  Column j of block (p, q) is the window |o_a| <= W of the PSF
// images around the lattice corners c of j, shifted to j and weighted with
// the multilinear weights of j between its corners (eq. trilinear; bilinear
// in 2D):  H_pq[j + o, j] = sum_c w_c(j) P[q][p][c + o], where j + o and c + o
// lie in the grid.  Per axis, the corners and the weight of every coordinate
// come from a small table (c0, c1, w) built on the host.
//
// Both products are gathers over the window of one output point (one thread
// per point, FP32 accumulation in a fixed order):
//   y = H x   : y_p[i] = sum_o sum_q x_q[i - o] sum_c w_c(i - o) P[q][p][c(i - o) + o]
//   y = H^T x : y_q[j] = sum_o sum_p x_p[j + o] sum_c w_c(j) P[q][p][c(j) + o]
// mono = 1 keeps the lnIp block (vectors of one parameter).
#include "common.h"
#include "kernels.h"

namespace lsrtm {

namespace {

// Corners and weight of coordinate j along axis a.
struct Cell {
    int c0, c1;
    float w;
};

__device__ __forceinline__ Cell cell_of(const PsfArgs& a, int ax, int j) {
    const int* t = a.tab + 3 * a.off[ax];
    Cell c;
    c.c0 = t[3 * j];
    c.c1 = t[3 * j + 1];
    c.w = __int_as_float(t[3 * j + 2]);
    return c;
}

// Sum over the 2^ndim corners of w_c * P[q][p][c + o] for the blocks in use;
// out[p][q] (mono: out[0][0] is the lnIp block).
__device__ __forceinline__ void corner_sum(const PsfArgs& a, const Cell (&cl)[3], int oz, int ox, int oy,
                                           float (&out)[2][2]) {
    const int nb = a.mono ? 1 : 2;
    for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q) out[p][q] = 0.f;
    const int ncorner = a.ndim == 3 ? 8 : 4;
    for (int m = 0; m < ncorner; ++m) {
        const int bz = m & 1, bx = (m >> 1) & 1, by = (m >> 2) & 1;
        const float wz = bz ? cl[0].w : 1.f - cl[0].w;
        const float wx = bx ? cl[1].w : 1.f - cl[1].w;
        const float wy = a.ndim == 3 ? (by ? cl[2].w : 1.f - cl[2].w) : 1.f;
        const float wgt = (wz * wx) * wy;
        if (wgt == 0.f) continue;
        const int sz = (bz ? cl[0].c1 : cl[0].c0) + oz;
        const int sx = (bx ? cl[1].c1 : cl[1].c0) + ox;
        const int sy = a.ndim == 3 ? (by ? cl[2].c1 : cl[2].c0) + oy : 0;
        if ((unsigned)sz >= (unsigned)a.n[0] || (unsigned)sx >= (unsigned)a.n[1] ||
            (unsigned)sy >= (unsigned)a.n[2])
            continue;
        const long long s = sz + (long long)a.n[0] * (sx + (long long)a.n[1] * sy);
        for (int p = 0; p < nb; ++p)
            for (int q = 0; q < nb; ++q) {
                // blocks stored [q][p][N]; mono reads the (1, 1) block
                const int qq = a.mono ? 1 : q, pp = a.mono ? 1 : p;
                out[p][q] = fmaf(wgt, a.psf[((long long)qq * 2 + pp) * a.N + s], out[p][q]);
            }
    }
}

__global__ void k_psf_apply(PsfArgs a, const float* __restrict__ x, float* __restrict__ y, int transpose) {
    const long long N = a.N;
    const int nb = a.mono ? 1 : 2;
    const int Wy = a.ndim == 3 ? a.W : 0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
         i += (long long)gridDim.x * blockDim.x) {
        const int iz = (int)(i % a.n[0]);
        const long long r = i / a.n[0];
        const int ix = (int)(r % a.n[1]);
        const int iy = (int)(r / a.n[1]);
        float acc[2] = {0.f, 0.f};
        Cell cl[3];
        if (transpose) {
            cl[0] = cell_of(a, 0, iz);
            cl[1] = cell_of(a, 1, ix);
            cl[2] = a.ndim == 3 ? cell_of(a, 2, iy) : Cell{0, 0, 0.f};
        }
        for (int oy = -Wy; oy <= Wy; ++oy)
            for (int ox = -a.W; ox <= a.W; ++ox)
                for (int oz = -a.W; oz <= a.W; ++oz) {
                    // forward: source point j = i - o; transpose: partner i + o
                    const int sgn = transpose ? 1 : -1;
                    const int jz = iz + sgn * oz, jx = ix + sgn * ox, jy = iy + sgn * oy;
                    if ((unsigned)jz >= (unsigned)a.n[0] || (unsigned)jx >= (unsigned)a.n[1] ||
                        (unsigned)jy >= (unsigned)a.n[2])
                        continue;
                    if (!transpose) {
                        cl[0] = cell_of(a, 0, jz);
                        cl[1] = cell_of(a, 1, jx);
                        cl[2] = a.ndim == 3 ? cell_of(a, 2, jy) : Cell{0, 0, 0.f};
                    }
                    float hs[2][2];
                    corner_sum(a, cl, oz, ox, oy, hs);
                    const long long jl = jz + (long long)a.n[0] * (jx + (long long)a.n[1] * jy);
                    for (int u = 0; u < nb; ++u) {
                        const float xv = x[u * N + jl];
                        for (int v = 0; v < nb; ++v) {
                            // forward: y_p += H_pq x_q (u = q, v = p);
                            // transpose: y_q += H_pq x_p (u = p, v = q)
                            const float hv = transpose ? hs[u][v] : hs[v][u];
                            acc[v] = fmaf(hv, xv, acc[v]);
                        }
                    }
                }
        for (int v = 0; v < nb; ++v) y[v * N + i] = acc[v];
    }
}

}  // namespace

hipError_t launch_psf_apply(const PsfArgs& a, const float* x, float* y, int transpose, hipStream_t st) {
    long long nb = (a.N + NTHREADS - 1) / NTHREADS;
    if (nb > 65536) nb = 65536;
    if (nb < 1) nb = 1;
    k_psf_apply<<<(int)nb, NTHREADS, 0, st>>>(a, x, y, transpose);
    return hipGetLastError();
}

// Unit spikes of parameter q on the scatterer lattice (all other entries of
// the [2][N] model vector zero).
__global__ void k_psf_spikes(PsfArgs a, int q, float* __restrict__ dm) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < 2 * a.N;
         i += (long long)gridDim.x * blockDim.x) {
        const int par = (int)(i / a.N);
        const long long g = i % a.N;
        const int iz = (int)(g % a.n[0]);
        const long long r = g / a.n[0];
        const int ix = (int)(r % a.n[1]);
        const int iy = (int)(r / a.n[1]);
        auto on = [&](int ax, int j) {
            // a lattice node is its own first corner with weight 0
            const Cell c = cell_of(a, ax, j);
            return (c.c0 == j && c.w == 0.f) || (c.c1 == j && c.w == 1.f);
        };
        const bool spike = par == q && on(0, iz) && on(1, ix) && (a.ndim == 2 || on(2, iy));
        dm[i] = spike ? 1.f : 0.f;
    }
}

hipError_t launch_psf_spikes(const PsfArgs& a, int q, float* dm, hipStream_t st) {
    long long nb = (2 * a.N + NTHREADS - 1) / NTHREADS;
    if (nb > 65536) nb = 65536;
    k_psf_spikes<<<(int)nb, NTHREADS, 0, st>>>(a, q, dm);
    return hipGetLastError();
}

}  // namespace lsrtm
