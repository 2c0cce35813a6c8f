// Auxiliary kernels: model preparation, receivers, image reduction,
// checkpoints and FP64 vector algebra.
#include <hip/hip_fp16.h>
#include <float.h>
#include "kernels.h"

namespace lsrtm {

static inline int nblocks(long long n, int per = NTHREADS) {
    long long b = (n + per - 1) / per;
    return (int)(b > 65535LL * 64 ? 65535LL * 64 : b);
}

__global__ void k_fill(float* __restrict__ p, long long n, float v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill64(double* __restrict__ p, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

hipError_t launch_fill(float* p, long long n, float v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_fill<<<nblocks(n), NTHREADS, 0, st>>>(p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_fill64<<<nblocks(n), NTHREADS, 0, st>>>(p, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Model and perturbation on a shot's padded grid
// ---------------------------------------------------------------------------
__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ double lnrho_at(const PrepArgs& a, int pz, int px, int py) {
    // padded coordinate -> physical global coordinate with edge replication
    const int z = a.lo[0] + clampi(pz - a.npml, 0, a.wn[0] - 1);
    const int x = a.lo[1] + clampi(px - a.npml, 0, a.wn[1] - 1);
    const int y = a.ndim == 3 ? a.lo[2] + clampi(py - a.npml, 0, a.wn[2] - 1) : 0;
    const long long g = z + (long long)a.gn[0] * (x + (long long)a.gn[1] * y);
    return (double)a.lnip[g] - (double)a.lnvp[g];
}

// sqrt(dt) * exp(-lnrho / 2), rounded to FP32 (the one rounding every user of
// sb and bdt shares)
__device__ __forceinline__ float sb_of(double dt, double lr) { return (float)(sqrt(dt) * exp(-0.5 * lr)); }

__global__ void k_model_prep(PrepArgs a) {
    const long long tot = (long long)a.N[0] * a.N[1] * a.N[2];
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
         e += (long long)gridDim.x * blockDim.x) {
        const int pz = (int)(e % a.N[0]);
        const long long r = e / a.N[0];
        const int px = (int)(r % a.N[1]);
        const int py = (int)(r / a.N[1]);
        const long long i = pz + a.sx * px + a.sy * py;
        const int z = a.lo[0] + clampi(pz - a.npml, 0, a.wn[0] - 1);
        const int x = a.lo[1] + clampi(px - a.npml, 0, a.wn[1] - 1);
        const int y = a.ndim == 3 ? a.lo[2] + clampi(py - a.npml, 0, a.wn[2] - 1) : 0;
        const long long g = z + (long long)a.gn[0] * (x + (long long)a.gn[1] * y);
        const double lk = (double)a.lnvp[g] + (double)a.lnip[g];
        a.kdt[i] = (float)(a.dt * exp(lk));
        const double lr = (double)a.lnip[g] - (double)a.lnvp[g];
        const float s0 = sb_of(a.dt, lr);
        a.sb[i] = s0;
        // dt b_a at the half node: the FP32 product the velocity kernels form
        const int pn[3] = {pz, px, py};
        for (int ax = 0; ax < a.ndim && a.bdt[0]; ++ax) {
            int q[3] = {pn[0], pn[1], pn[2]};
            q[ax] = q[ax] + 1 < a.N[ax] ? q[ax] + 1 : q[ax];
            a.bdt[ax][i] = s0 * sb_of(a.dt, lnrho_at(a, q[0], q[1], q[2]));
        }
    }
}

hipError_t launch_model_prep(const PrepArgs& a, hipStream_t st) {
    const long long tot = (long long)a.N[0] * a.N[1] * a.N[2];
    k_model_prep<<<nblocks(tot), NTHREADS, 0, st>>>(a);
    return hipGetLastError();
}

__global__ void k_dm_prep(DmArgs a) {
    const long long tot = (long long)a.N[0] * a.N[1] * a.N[2];
    const int ndim = a.ndim;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
         e += (long long)gridDim.x * blockDim.x) {
        const int pz = (int)(e % a.N[0]);
        const long long r = e / a.N[0];
        const int px = (int)(r % a.N[1]);
        const int py = (int)(r / a.N[1]);
        const long long i = pz + a.sx * px + a.sy * py;
        const int z = pz - a.npml, x = px - a.npml, y = ndim == 3 ? py - a.npml : 0;
        float dr = 0.f, dk = 0.f;
        if (z >= 0 && z < a.wn[0] && x >= 0 && x < a.wn[1] && (ndim == 2 || (y >= 0 && y < a.wn[2]))) {
            const long long g = (a.lo[0] + z) +
                                (long long)a.gn[0] * ((a.lo[1] + x) + (long long)a.gn[1] * (ndim == 3 ? a.lo[2] + y : 0));
            const float m1 = a.dm[g], m2 = a.dm[a.gpts + g];
            dr = m2 - m1;
            dk = m2 + m1;
        }
        a.dlnr[i] = dr;
        a.dlnk[i] = dk;
    }
}

hipError_t launch_dm_prep(const DmArgs& a, hipStream_t st) {
    const long long tot = (long long)a.N[0] * a.N[1] * a.N[2];
    k_dm_prep<<<nblocks(tot), NTHREADS, 0, st>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Receivers
// ---------------------------------------------------------------------------
__global__ void k_gather(const Slot* __restrict__ slots, const Rec* __restrict__ rec, int nrec, int n,
                         int from_scattered, float* __restrict__ d) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrec) return;
    const Rec R = rec[r];
    const DSlot& S = dev_slots(slots)[R.slot];
    const gfloat* f = from_scattered ? S.q : S.p;
    d[R.out + (long long)n * R.stride] = f[R.idx];
}

hipError_t launch_gather(const Slot* slots, const Rec* rec, int nrec, int n, int from_scattered,
                         float* d, hipStream_t st) {
    if (nrec <= 0) return hipSuccess;
    k_gather<<<(nrec + NTHREADS - 1) / NTHREADS, NTHREADS, 0, st>>>(slots, rec, nrec, n, from_scattered, d);
    return hipGetLastError();
}

__global__ void k_inject(const Slot* __restrict__ slots, const int* __restrict__ node_slot,
                         const int* __restrict__ node_idx, const int* __restrict__ node_ptr,
                         const Rec* __restrict__ rec, int nnode, int n, const float* __restrict__ d) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= nnode) return;
    float s = 0.f;
    for (int r = node_ptr[u]; r < node_ptr[u + 1]; ++r) s = s + d[rec[r].out + (long long)n * rec[r].stride];
    const DSlot& S = dev_slots(slots)[node_slot[u]];
    gfloat* q = S.q;
    const int i = node_idx[u];
    // the field holds Q = -dt kappa p~, so the source added to p~ enters as
    // -dt kappa s
    q[i] = q[i] - S.kdt[i] * s;
}

hipError_t launch_inject(const Slot* slots, const int* node_slot, const int* node_idx,
                         const int* node_ptr, const Rec* rec, int nnode, int n, const float* d,
                         hipStream_t st) {
    if (nnode <= 0) return hipSuccess;
    k_inject<<<(nnode + NTHREADS - 1) / NTHREADS, NTHREADS, 0, st>>>(slots, node_slot, node_idx, node_ptr,
                                                                     rec, nnode, n, d);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Images
// ---------------------------------------------------------------------------
__global__ void k_image_reduce(ImgArgs a) {
    const int ndim = a.ndim;
    for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < a.gpts;
         g += (long long)gridDim.x * blockDim.x) {
        const int z = (int)(g % a.gn[0]);
        const long long r = g / a.gn[0];
        const int x = (int)(r % a.gn[1]);
        const int y = (int)(r / a.gn[1]);
        double m1 = a.acc[g], m2 = a.acc[a.gpts + g];
        for (int s = 0; s < a.nslot; ++s) {
            const int* w = a.win + 6 * s;
            if (z < w[0] || z >= w[1] || x < w[2] || x >= w[3]) continue;
            if (ndim == 3 && (y < w[4] || y >= w[5])) continue;
            const DSlot& S = dev_slots(a.slots)[s];
            const long long i = (z - w[0] + a.npml) + S.sx * (x - w[2] + a.npml) +
                                (ndim == 3 ? S.sy * (long long)(y - w[4] + a.npml) : 0LL);
            const double gr = S.gr[i], gk = S.gk[i];
            m1 += -gr + gk;
            m2 += gr + gk;
        }
        a.acc[g] = m1;
        a.acc[a.gpts + g] = m2;
    }
}

hipError_t launch_image_reduce(const ImgArgs& a, hipStream_t st) {
    k_image_reduce<<<nblocks(a.gpts), NTHREADS, 0, st>>>(a);
    return hipGetLastError();
}

__global__ void k_image_store(const double* __restrict__ acc, float* __restrict__ img, long long n, int accumulate) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        img[i] = accumulate ? (float)((double)img[i] + acc[i]) : (float)acc[i];
}

hipError_t launch_image_store(const double* acc, float* img, long long n, int accumulate, hipStream_t st) {
    k_image_store<<<nblocks(n), NTHREADS, 0, st>>>(acc, img, n, accumulate);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pseudo-Hessian (appendix B of the paper)
// ---------------------------------------------------------------------------
// Per physical node, in shot order: the slots' time sums of the squared
// velocity increments (w_a, at half nodes) moved onto the node with the
// squared weights of the half-node average -- 1/4 from each neighbouring
// half node, weight 1 from a clamped last half node onto its own node -- into
// acc[0], and the time sums of q^2 (g_kappa) into acc[1].
__global__ void k_ph_reduce(ImgArgs a) {
    const int ndim = a.ndim;
    for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < a.gpts;
         g += (long long)gridDim.x * blockDim.x) {
        const int z = (int)(g % a.gn[0]);
        const long long r = g / a.gn[0];
        const int x = (int)(r % a.gn[1]);
        const int y = (int)(r / a.gn[1]);
        double hv = a.acc[g], hq = a.acc[a.gpts + g];
        for (int s = 0; s < a.nslot; ++s) {
            const int* w = a.win + 6 * s;
            if (z < w[0] || z >= w[1] || x < w[2] || x >= w[3]) continue;
            if (ndim == 3 && (y < w[4] || y >= w[5])) continue;
            const DSlot& S = dev_slots(a.slots)[s];
            const int c[3] = {z - w[0] + a.npml, x - w[2] + a.npml, ndim == 3 ? y - w[4] + a.npml : 0};
            const long long i = c[0] + S.sx * c[1] + S.sy * (long long)c[2];
            for (int ax = 0; ax < ndim; ++ax) {
                const long long stride = ax == 0 ? 1LL : (ax == 1 ? S.sx : S.sy);
                const double v = S.w[ax][i];
                double t = 0.25 * v;
                if (c[ax] > 0) t += 0.25 * (double)S.w[ax][i - stride];
                if (c[ax] == S.n[ax] - 1) t += 0.75 * v;
                hv += t;
            }
            hq += S.gk[i];
        }
        a.acc[g] = hv;
        a.acc[a.gpts + g] = hq;
    }
}

hipError_t launch_ph_reduce(const ImgArgs& a, hipStream_t st) {
    k_ph_reduce<<<nblocks(a.gpts), NTHREADS, 0, st>>>(a);
    return hipGetLastError();
}

// h = rho^2 / dt * acc[0] + (dt kappa)^2 / dt * acc[1], rho and kappa from
// the physical model logs (lnrho = lnIp - lnVp, lnkappa = lnIp + lnVp).
__global__ void k_ph_finish(const double* __restrict__ acc, const float* __restrict__ lnvp,
                            const float* __restrict__ lnip, double dt, float* __restrict__ h, long long n) {
    for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < n;
         g += (long long)gridDim.x * blockDim.x) {
        const double lv = lnvp[g], li = lnip[g];
        const double rho2 = exp(2.0 * (li - lv));
        const double dk = dt * exp(li + lv);
        h[g] = (float)((rho2 * acc[g] + dk * dk * acc[n + g]) / dt);
    }
}

hipError_t launch_ph_finish(const double* acc, const float* lnvp, const float* lnip, double dt, float* h,
                            long long n, hipStream_t st) {
    k_ph_finish<<<nblocks(n), NTHREADS, 0, st>>>(acc, lnvp, lnip, dt, h, n);
    return hipGetLastError();
}

// minv[0][g] = minv[1][g] = 1 / (h[g] + eps): the same diagonal for lnVp and lnIp.
__global__ void k_ph_minv(const float* __restrict__ h, double eps, float* __restrict__ minv, long long n) {
    for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < n;
         g += (long long)gridDim.x * blockDim.x) {
        const float m = (float)(1.0 / ((double)h[g] + eps));
        minv[g] = m;
        minv[n + g] = m;
    }
}

hipError_t launch_ph_minv(const float* h, double eps, float* minv, long long n, hipStream_t st) {
    k_ph_minv<<<nblocks(n), NTHREADS, 0, st>>>(h, eps, minv, n);
    return hipGetLastError();
}

// out = a * b elementwise (the diagonal preconditioner applied to a vector).
__global__ void k_mul(const float* __restrict__ a, const float* __restrict__ b, float* __restrict__ out,
                      long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        out[i] = a[i] * b[i];
}

hipError_t launch_mul(const float* a, const float* b, float* out, long long n, hipStream_t st) {
    k_mul<<<nblocks(n), NTHREADS, 0, st>>>(a, b, out, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Top mute of recorded data (the nonlinear-residual data preparation)
// ---------------------------------------------------------------------------
// Receiver j's trace starts at d + off[j] with stride stride[j]; sample n is
// recorded at time (n + 1) dt.  Samples before tc[j] are zeroed, the next
// ntaper samples ramp up with 0.5 (1 - cos(pi (t - tc) / (ntaper dt))).
__global__ void k_mute(float* __restrict__ d, const long long* __restrict__ off, const int* __restrict__ stride,
                       const double* __restrict__ tc, int nrec, int nt, double dt, int ntaper) {
    const long long total = (long long)nrec * nt;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(e % nrec);
        const int n = (int)(e / nrec);
        const double t = (n + 1) * dt;
        double wgt = 1.0;
        if (t < tc[j]) wgt = 0.0;
        else if (ntaper > 0 && t < tc[j] + ntaper * dt) wgt = 0.5 * (1.0 - cos(M_PI * (t - tc[j]) / (ntaper * dt)));
        if (wgt != 1.0) {
            float* p = d + off[j] + (long long)n * stride[j];
            *p = (float)(wgt * (double)*p);
        }
    }
}

// Per-receiver tables of the mute from the device-resident acquisition of a
// launch group: the trace offset and row length of receiver j (its Rec
// entry) and its cut time tc = t0 + |x_r - x_s| / v_mute, the distance taken
// from the padded-grid coordinates of the receiver and of its shot's source
// (the padding cancels), summed over the axes in the order z, x, y.
__global__ void k_mute_tables(const DSlot* __restrict__ slots, const Rec* __restrict__ rec, int nrec, int ndim,
                              double hz, double hx, double hy, double t0, double v_mute, long long* __restrict__ off,
                              int* __restrict__ stride, double* __restrict__ tc) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nrec) return;
    const Rec R = rec[j];
    const DSlot& S = slots[R.slot];
    const long long ldz = S.ldz, nx = S.n[1];
    const long long ir = R.idx, is = S.src;
    const double h[3] = {hz, hx, hy};
    const long long cr[3] = {ir % ldz, (ir / ldz) % nx, ir / (ldz * nx)};
    const long long cs[3] = {is % ldz, (is / ldz) % nx, is / (ldz * nx)};
    double d2 = 0.0;
    for (int a = 0; a < ndim; ++a) {
        const double x = (double)(cr[a] - cs[a]) * h[a];
        d2 = d2 + x * x;
    }
    off[j] = R.out;
    stride[j] = R.stride;
    tc[j] = t0 + sqrt(d2) / v_mute;
}

hipError_t launch_mute_tables(const Slot* slots, const Rec* rec, int nrec, int ndim, const double* h, double t0,
                              double v_mute, long long* off, int* stride, double* tc, hipStream_t st) {
    if (nrec <= 0) return hipSuccess;
    k_mute_tables<<<(nrec + NTHREADS - 1) / NTHREADS, NTHREADS, 0, st>>>(dev_slots(slots), rec, nrec, ndim, h[0], h[1],
                                                                         h[2], t0, v_mute, off, stride, tc);
    return hipGetLastError();
}

hipError_t launch_mute(float* d, const long long* off, const int* stride, const double* tc, int nrec, int nt,
                       double dt, int ntaper, hipStream_t st) {
    if (nrec <= 0 || nt <= 0) return hipSuccess;
    k_mute<<<nblocks((long long)nrec * nt), NTHREADS, 0, st>>>(d, off, stride, tc, nrec, nt, dt, ntaper);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reductions (fixed-shape trees, deterministic)
// ---------------------------------------------------------------------------
template <typename T, typename Op>
__device__ T block_reduce(T v, Op op) {
    __shared__ T sh[NTHREADS / 64];
    for (int o = 32; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o, 64));
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    if (w == 0) {
        // only lanes 0..3 carry data; the xor butterfly below stays within them
        v = lane < NTHREADS / 64 ? sh[lane] : sh[0];
        for (int o = 2; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o, 64));
    }
    return v;
}

struct MaxOp { __device__ float operator()(float a, float b) const { return fmaxf(a, b); } };
struct AddOp { __device__ double operator()(double a, double b) const { return a + b; } };

__device__ __forceinline__ float absfin(float x) {
    const float v = fabsf(x);
    return (v <= FLT_MAX) ? v : INFINITY;   // NaN and Inf map to +inf
}

__global__ void k_maxabs(const float* __restrict__ x, long long n, float* __restrict__ partial) {
    float m = 0.f;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        m = fmaxf(m, absfin(x[i]));
    m = block_reduce(m, MaxOp());
    if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

hipError_t launch_maxabs(const float* x, long long n, float* partial, int nblk, hipStream_t st) {
    k_maxabs<<<nblk, NTHREADS, 0, st>>>(x, n, partial);
    return hipGetLastError();
}

// Largest value of x (NaN or Inf anywhere -> +inf).
__global__ void k_maxval(const float* __restrict__ x, long long n, float* __restrict__ partial) {
    float m = -FLT_MAX;
    bool bad = false;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const float v = x[i];
        bad = bad || !(fabsf(v) <= FLT_MAX);
        m = fmaxf(m, v);
    }
    if (bad) m = INFINITY;
    m = block_reduce(m, MaxOp());
    if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

hipError_t launch_maxval(const float* x, long long n, float* partial, int nblk, hipStream_t st) {
    k_maxval<<<nblk, NTHREADS, 0, st>>>(x, n, partial);
    return hipGetLastError();
}

__global__ void k_dot_partial(const float* __restrict__ a, const float* __restrict__ b, long long n,
                              double* __restrict__ partial) {
    double s = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        s += (double)a[i] * (double)b[i];
    s = block_reduce(s, AddOp());
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void k_dot_final(const double* __restrict__ partial, int nblk, double* __restrict__ out) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) s += partial[i];
    s = block_reduce(s, AddOp());
    if (threadIdx.x == 0) out[0] = s;
}

hipError_t launch_dot(const float* a, const float* b, long long n, double* partial, int nblk,
                      double* out, hipStream_t st) {
    k_dot_partial<<<nblk, NTHREADS, 0, st>>>(a, b, n, partial);
    k_dot_final<<<1, NTHREADS, 0, st>>>(partial, nblk, out);
    return hipGetLastError();
}

__global__ void k_axpy(double alpha, const float* __restrict__ x, float* __restrict__ y, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        y[i] = (float)((double)y[i] + alpha * (double)x[i]);
}
__global__ void k_xpby(const float* __restrict__ x, double beta, float* __restrict__ y, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        y[i] = (float)((double)x[i] + beta * (double)y[i]);
}
__global__ void k_copy(const float* __restrict__ x, float* __restrict__ y, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        y[i] = x[i];
}

hipError_t launch_axpy(double alpha, const float* x, float* y, long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_axpy<<<nblocks(n), NTHREADS, 0, st>>>(alpha, x, y, n);
    return hipGetLastError();
}
hipError_t launch_xpby(const float* x, double beta, float* y, long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_xpby<<<nblocks(n), NTHREADS, 0, st>>>(x, beta, y, n);
    return hipGetLastError();
}
hipError_t launch_copy(const float* x, float* y, long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_copy<<<nblocks(n), NTHREADS, 0, st>>>(x, y, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Calibration: streaming rate of a mix of arrays like the stencil kernels'
// ---------------------------------------------------------------------------
struct MixArrays {
    float* a[16];
};

// Every element of arrays 0 .. NR-1 read once, of arrays NR .. NR+NW-1
// written once (the sum of the reads times the array's rank, so that no load
// is dead), walking the elements in order.
template <int NR, int NW>
__global__ void __launch_bounds__(NTHREADS) k_mix_flat(MixArrays A, long long n) {
    for (long long i = blockIdx.x * (long long)NTHREADS + threadIdx.x; i < n; i += (long long)gridDim.x * NTHREADS) {
        float s = 0.f;
#pragma unroll
        for (int k = 0; k < NR; ++k) s += A.a[k][i];
#pragma unroll
        for (int k = 0; k < NW; ++k) A.a[NR + k][i] = s * (float)(k + 1);
    }
}

// The same, walking the elements as the 3D stencil tiles do: a block owns a
// column of 64 x 4 nodes of an nz x nx x ny grid (z stride ldz) and marches
// 32 planes along y; blocks are remapped onto the XCDs as the tiles are.
template <int NR, int NW>
__global__ void __launch_bounds__(NTHREADS) k_mix_march(MixArrays A, int nz, int nx, int ny, int ldz) {
    const int ntz = (nz + 63) / 64, ntx = (nx + 3) / 4;
    int b = xcd_remap(blockIdx.x, gridDim.x);
    const int tz = b % ntz;
    b /= ntz;
    const int tx = b % ntx;
    const int y0 = (b / ntx) * 32, y1 = min(y0 + 32, ny);
    const int z = tz * 64 + (int)threadIdx.x % 64, x = tx * 4 + (int)threadIdx.x / 64;
    if (z >= nz || x >= nx) return;
    for (int y = y0; y < y1; ++y) {
        const long long i = ((long long)y * nx + x) * ldz + z;
        float s = 0.f;
#pragma unroll
        for (int k = 0; k < NR; ++k) s += A.a[k][i];
#pragma unroll
        for (int k = 0; k < NW; ++k) A.a[NR + k][i] = s * (float)(k + 1);
    }
}

template <int NR, int NW>
static hipError_t mix_t(float* buf, long long n, const int* grid, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    MixArrays A;
    for (int k = 0; k < 16; ++k) A.a[k] = buf + (long long)(k < NR + NW ? k : 0) * n;
    if (!grid) {
        launch_k(k_mix_flat<NR, NW>, dim3(nblocks(n)), dim3(NTHREADS), st, e0, e1, A, n);
    } else {
        const long long nb = (long long)((grid[0] + 63) / 64) * ((grid[1] + 3) / 4) * ((grid[2] + 31) / 32);
        launch_k(k_mix_march<NR, NW>, dim3((unsigned)nb), dim3(NTHREADS), st, e0, e1, A, grid[0], grid[1],
                 grid[2], grid[3]);
    }
    return hipGetLastError();
}

hipError_t launch_stream_mix(float* buf, long long n, int nread, int nwrite, const int* grid, hipStream_t st,
                             hipEvent_t e0, hipEvent_t e1) {
    const int key = nread * 16 + nwrite;
    switch (key) {
    case 10 * 16 + 6: return mix_t<10, 6>(buf, n, grid, st, e0, e1);
    case 10 * 16 + 2: return mix_t<10, 2>(buf, n, grid, st, e0, e1);
    case 5 * 16 + 6: return mix_t<5, 6>(buf, n, grid, st, e0, e1);
    case 5 * 16 + 2: return mix_t<5, 2>(buf, n, grid, st, e0, e1);
    case 2 * 16 + 1: return mix_t<2, 1>(buf, n, grid, st, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Checkpoints
// ---------------------------------------------------------------------------
// Field f of a slot: 0 = p, 1 + a = v_a.
__device__ __forceinline__ gfloat* slot_field(const DSlot& S, int f) { return f == 0 ? S.p : S.v[f - 1]; }

// Strip element e of axis a -> linear index (z, x, y layout with strides).
__device__ __forceinline__ long long strip_index(const DSlot& S, int ndim, int a, int Sd, long long e) {
    const int nz = S.n[0], nx = S.n[1];
    const int Sa = Sd < S.n[a] ? Sd : S.n[a];
    int c[3] = {0, 0, 0};
    // layout: axis-a coordinate (2*Sa values) is the fastest after z for
    // a != 0; for a = 0 it is the fastest of all.
    if (a == 0) {
        const int r = (int)(e % (2 * Sa));
        long long t = e / (2 * Sa);
        c[0] = r < Sa ? r : nz - Sa + (r - Sa);
        c[1] = (int)(t % nx);
        c[2] = (int)(t / nx);
    } else if (a == 1) {
        c[0] = (int)(e % nz);
        long long t = e / nz;
        const int r = (int)(t % (2 * Sa));
        c[1] = r < Sa ? r : nx - Sa + (r - Sa);
        c[2] = (int)(t / (2 * Sa));
    } else {
        c[0] = (int)(e % nz);
        long long t = e / nz;
        c[1] = (int)(t % nx);
        const int r = (int)(t / nx);
        c[2] = r < Sa ? r : S.n[2] - Sa + (r - Sa);
    }
    return c[0] + S.sx * c[1] + S.sy * c[2];
}

__device__ __forceinline__ long long strip_count(const DSlot& S, int a, int Sd) {
    const int Sa = Sd < S.n[a] ? Sd : S.n[a];
    long long c = 2LL * Sa;
    for (int b = 0; b < 3; ++b)
        if (b != a) c *= S.n[b];
    return c;
}

using gu16 = __attribute__((address_space(1))) unsigned short;

__device__ __forceinline__ unsigned short f2bf_rne(float x) {
    unsigned int u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float(((unsigned int)b) << 16); }

// grid: (blocks, 1 + ndim, nslot); partial max |x| per block.
__global__ void k_ckpt_maxabs(CkptArgs a) {
    const DSlot& S = dev_slots(a.slots)[blockIdx.z];
    const gfloat* f = slot_field(S, blockIdx.y);
    float m = 0.f;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < S.npts;
         i += (long long)gridDim.x * blockDim.x)
        m = fmaxf(m, absfin(f[i]));
    m = block_reduce(m, MaxOp());
    if (threadIdx.x == 0) a.partial[((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = m;
}

// grid: (1, 1 + ndim, nslot)
__global__ void k_ckpt_scale(CkptArgs a) {
    float m = 0.f;
    const long long base = ((long long)blockIdx.z * gridDim.y + blockIdx.y) * a.nblk;
    for (int i = threadIdx.x; i < a.nblk; i += blockDim.x) m = fmaxf(m, a.partial[base + i]);
    m = block_reduce(m, MaxOp());
    if (threadIdx.x == 0) {
        if (!(m <= FLT_MAX)) a.nonfinite[0] = 1;
        float s = 1.f;
        if (a.dtype == 1) s = m / 16384.f;       // FP16: |x/s| <= 2^14
        else if (a.dtype == 2) s = m;            // BF16: |x/s| <= 1
        a.scales[blockIdx.z * (1 + a.ndim) + blockIdx.y] = s;
    }
}

// grid: (blocks, 1 + ndim, nslot): pack the fields.
__global__ void k_ckpt_pack(CkptArgs a) {
    const DSlot& S = dev_slots(a.slots)[blockIdx.z];
    const int f = blockIdx.y;
    const gfloat* src = slot_field(S, f);
    gchar* base = S.ck + (long long)(a.j - 1) * S.ckbytes;
    const float s = a.scales[blockIdx.z * (1 + a.ndim) + f];
    const float inv = s > 0.f ? 1.f / s : 0.f;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < S.npts;
         i += (long long)gridDim.x * blockDim.x) {
        const float x = src[i];
        if (a.dtype == 0) {
            reinterpret_cast<gfloat*>(base)[f * S.npts + i] = x;
        } else if (a.dtype == 1) {
            reinterpret_cast<gu16*>(base)[f * S.npts + i] = __half_as_ushort(__float2half_rn(x * inv));
        } else {
            reinterpret_cast<gu16*>(base)[f * S.npts + i] = f2bf_rne(x * inv);
        }
    }
}

__global__ void k_ckpt_unpack(CkptArgs a) {
    const DSlot& S = dev_slots(a.slots)[blockIdx.z];
    const int f = blockIdx.y;
    gfloat* dst = slot_field(S, f);
    const gchar* base = S.ck + (long long)(a.j - 1) * S.ckbytes;
    const float s = a.scales[blockIdx.z * (1 + a.ndim) + f];
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < S.npts;
         i += (long long)gridDim.x * blockDim.x) {
        float x;
        if (a.dtype == 0) x = reinterpret_cast<const gfloat*>(base)[f * S.npts + i];
        else if (a.dtype == 1) x = __half2float(__ushort_as_half(reinterpret_cast<const gu16*>(base)[f * S.npts + i])) * s;
        else x = bf2f(reinterpret_cast<const gu16*>(base)[f * S.npts + i]) * s;
        dst[i] = x;
    }
}

// grid: (blocks, 2 * ndim, nslot): CPML memories of the strips, FP32.
// Memory m: psi_a for m = 2a, phi_a for m = 2a + 1.
template <bool SAVE>
__global__ void k_ckpt_strips(CkptArgs a) {
    const DSlot& S = dev_slots(a.slots)[blockIdx.z];
    const int m = blockIdx.y, ax = m >> 1;
    gfloat* f = (m & 1) ? S.phi[ax] : S.psi[ax];
    const int esz = a.dtype == 0 ? 4 : 2;
    long long off = (long long)(1 + a.ndim) * S.npts * esz;
    for (int mm = 0; mm < m; ++mm) off += strip_count(S, mm >> 1, a.S) * 4;
    gfloat* buf = reinterpret_cast<gfloat*>(S.ck + (long long)(a.j - 1) * S.ckbytes + off);
    const long long cnt = strip_count(S, ax, a.S);
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < cnt;
         e += (long long)gridDim.x * blockDim.x) {
        const long long i = strip_index(S, a.ndim, ax, a.S, e);
        if (SAVE) buf[e] = f[i];
        else f[i] = buf[e];
    }
}

static int grid_for(long long n) {
    long long b = (n + NTHREADS - 1) / NTHREADS;
    return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

hipError_t launch_ckpt_save(const CkptArgs& a, long long max_npts, hipStream_t st) {
    const int nf = 1 + a.ndim;
    k_ckpt_maxabs<<<dim3(a.nblk, nf, a.nslot), NTHREADS, 0, st>>>(a);
    k_ckpt_scale<<<dim3(1, nf, a.nslot), NTHREADS, 0, st>>>(a);
    k_ckpt_pack<<<dim3(grid_for(max_npts), nf, a.nslot), NTHREADS, 0, st>>>(a);
    k_ckpt_strips<true><<<dim3(grid_for(max_npts / 4 + 1), 2 * a.ndim, a.nslot), NTHREADS, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_ckpt_load(const CkptArgs& a, long long max_npts, hipStream_t st) {
    const int nf = 1 + a.ndim;
    k_ckpt_unpack<<<dim3(grid_for(max_npts), nf, a.nslot), NTHREADS, 0, st>>>(a);
    k_ckpt_strips<false><<<dim3(grid_for(max_npts / 4 + 1), 2 * a.ndim, a.nslot), NTHREADS, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace lsrtm
