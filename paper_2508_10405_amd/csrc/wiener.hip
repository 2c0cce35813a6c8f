// Nonstationary Wiener deblurring (appendix D of the paper).
//
// The Hessian is taken as locally translation invariant, hence diagonal in
// the Fourier basis of each local block.  Per block, with F its Fourier
// transform, the regularised inverse eigenvalues are
//   Lambda^-1 = conj(F m_blur) F m_ref / (|F m_blur|^2 + eps)
// and the block's estimate is F^-1 [Lambda^-1 F m_in] (eq. sol); eps is
// eps_rel times the block's largest |F m_blur|^2.  Blocks of `block` nodes
// per axis start every block/2 nodes from -block/2 and are tapered with
// sin^2(pi (u + 1/2) / block) per axis, so every node lies in 2^ndim blocks
// whose tapers add up to one; the estimates are merged with these valences,
// dm = sum_w dm_w / sum_w t_w.
//
// Steps: each image is scaled by its largest magnitude (the filter is
// invariant to the scale of m_ref and m_blur and linear in m_in, and migrated
// images can be small enough for |F m|^2 to leave the FP32 range), a gather
// kernel builds the tapered blocks of the three images (one batch of complex
// arrays), hipFFT transforms them, one workgroup per block forms the filtered
// spectrum, hipFFT transforms back, and a gather kernel merges the 2^ndim
// blocks over each node and restores the scale.
#include "common.h"
#include "kernels.h"
#include <hipfft/hipfft.h>

#include <cmath>
#include <vector>

namespace lsrtm {

struct WArgs {
    int n[3];          // image sizes (z, x, y); n[2] = 1 in 2D
    int ndim;
    int B;             // block size per axis
    int K[3];          // blocks per axis
    long long nwin;    // K[0] K[1] K[2]
    long long bs;      // B^ndim
    long long N;       // n[0] n[1] n[2]
    const float* taper;
    const float* scale;  // largest |value| of ref, blur, in
};

constexpr int NPART = 256;

struct WienerWork {
    int ndim = 0, n[3] = {0, 0, 0}, block = 0;
    long long nwin = 0, bs = 0;
    hipfftComplex* buf = nullptr;    // [3][nwin][bs]: ref, blur, in spectra
    float* taper = nullptr;          // [block]
    float* scale = nullptr;          // [NPART * 3] partial maxima, then the 3 scales
    hipfftHandle fwd = 0, inv = 0;
    bool plans = false;
};

namespace {

__device__ __forceinline__ void window_origin(const WArgs& a, long long w, int (&o)[3]) {
    const int h = a.B / 2;
    const int wz = (int)(w % a.K[0]);
    const long long r = w / a.K[0];
    const int wx = (int)(r % a.K[1]);
    const int wy = (int)(r / a.K[1]);
    o[0] = wz * h - h;
    o[1] = wx * h - h;
    o[2] = a.ndim == 3 ? wy * h - h : 0;
}

// Largest |value| of the three images: NPART partial maxima per image, then
// one workgroup reduces them into scale[0..2].
__global__ void k_w_maxabs(const float* __restrict__ ref, const float* __restrict__ blur,
                           const float* __restrict__ in, long long n, float* __restrict__ part) {
    __shared__ float red[NTHREADS];
    const float* img = blockIdx.y == 0 ? ref : (blockIdx.y == 1 ? blur : in);
    float m = 0.f;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(img[i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = NTHREADS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.y * NPART + blockIdx.x] = red[0];
}

__global__ void k_w_scale(float* __restrict__ part) {
    __shared__ float red[NTHREADS];
    for (int k = 0; k < 3; ++k) {
        red[threadIdx.x] = threadIdx.x < NPART ? part[k * NPART + threadIdx.x] : 0.f;
        __syncthreads();
        for (int s = NTHREADS / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
            __syncthreads();
        }
        if (threadIdx.x == 0) part[3 * NPART + k] = red[0];
        __syncthreads();
    }
}

__global__ void k_w_extract(WArgs a, const float* __restrict__ ref, const float* __restrict__ blur,
                            const float* __restrict__ in, hipfftComplex* __restrict__ buf) {
    const long long per = a.nwin * a.bs;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < 3 * per;
         e += (long long)gridDim.x * blockDim.x) {
        const int k = (int)(e / per);
        const long long r = e % per;
        const long long w = r / a.bs;
        const long long u = r % a.bs;
        int o[3];
        window_origin(a, w, o);
        const int uz = (int)(u % a.B);
        const int ux = (int)((u / a.B) % a.B);
        const int uy = a.ndim == 3 ? (int)(u / ((long long)a.B * a.B)) : 0;
        const int gz = o[0] + uz, gx = o[1] + ux, gy = o[2] + uy;
        float v = 0.f;
        if ((unsigned)gz < (unsigned)a.n[0] && (unsigned)gx < (unsigned)a.n[1] && (unsigned)gy < (unsigned)a.n[2]) {
            const long long g = gz + (long long)a.n[0] * (gx + (long long)a.n[1] * gy);
            const float* img = k == 0 ? ref : (k == 1 ? blur : in);
            float t = a.taper[uz] * a.taper[ux];
            if (a.ndim == 3) t *= a.taper[uy];
            const float sc = a.scale[k];
            v = sc > 0.f ? t * (img[g] / sc) : 0.f;
        }
        buf[e] = make_hipFloatComplex(v, 0.f);
    }
}

// One workgroup per block: the filtered spectrum Lambda^-1 F m_in / bs (the
// inverse transform is unnormalised) written over F m_ref.  The block's
// F m_blur is first divided by its largest component magnitude beta (blocks
// at the edge of the illumination can hold values whose squares leave the
// FP32 range), which leaves Lambda^-1 beta unchanged:
//   Lambda^-1 = conj(b') F m_ref / (|b'|^2 + eps_rel max |b'|^2) / beta,  b' = F m_blur / beta.
__device__ __forceinline__ float block_max(float v, float* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = NTHREADS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    const float r = red[0];
    __syncthreads();
    return r;
}

__global__ void k_w_filter(WArgs a, double eps_rel, hipfftComplex* __restrict__ buf) {
    __shared__ float red[NTHREADS];
    const long long w = blockIdx.x;
    hipfftComplex* A = buf + w * a.bs;
    const hipfftComplex* Bh = buf + (a.nwin + w) * a.bs;
    const hipfftComplex* C = buf + (2 * a.nwin + w) * a.bs;
    float m = 0.f;
    for (long long u = threadIdx.x; u < a.bs; u += NTHREADS) {
        const hipfftComplex b = Bh[u];
        m = fmaxf(m, fmaxf(fabsf(b.x), fabsf(b.y)));
    }
    const float beta = block_max(m, red);
    if (!(beta > 0.f)) {
        for (long long u = threadIdx.x; u < a.bs; u += NTHREADS) A[u] = make_hipFloatComplex(0.f, 0.f);
        return;
    }
    const float ib = 1.f / beta;
    float p = 0.f;
    for (long long u = threadIdx.x; u < a.bs; u += NTHREADS) {
        const hipfftComplex b = Bh[u];
        const float bx = b.x * ib, by = b.y * ib;
        p = fmaxf(p, bx * bx + by * by);
    }
    const float eps = (float)(eps_rel * (double)block_max(p, red));
    const float inv_bs = 1.f / (float)a.bs;
    for (long long u = threadIdx.x; u < a.bs; u += NTHREADS) {
        const hipfftComplex b = Bh[u], r = A[u], c = C[u];
        const float bx = b.x * ib, by = b.y * ib;
        const float den = (bx * bx + by * by) + eps;
        // conj(b') r / den / beta
        const float gx = ((bx * r.x + by * r.y) / den) * ib;
        const float gy = ((bx * r.y - by * r.x) / den) * ib;
        // (g c) / bs
        A[u] = make_hipFloatComplex((gx * c.x - gy * c.y) * inv_bs, (gx * c.y + gy * c.x) * inv_bs);
    }
}

__global__ void k_w_merge(WArgs a, const hipfftComplex* __restrict__ bufA, float* __restrict__ out) {
    const int h = a.B / 2;
    for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < a.N;
         g += (long long)gridDim.x * blockDim.x) {
        const int c[3] = {(int)(g % a.n[0]), (int)((g / a.n[0]) % a.n[1]),
                          (int)(g / ((long long)a.n[0] * a.n[1]))};
        float num = 0.f, den = 0.f;
        const int ncomb = a.ndim == 3 ? 8 : 4;
        for (int m = 0; m < ncomb; ++m) {
            long long w = 0, u = 0, wstride = 1, ustride = 1;
            float t = 1.f;
            bool ok = true;
            for (int ax = 0; ax < a.ndim; ++ax) {
                // blocks k = c/h and c/h + 1 start at (k - 1) h and cover c
                const int k = c[ax] / h + ((m >> ax) & 1);
                const int loc = c[ax] - (k * h - h);
                ok = ok && k < a.K[ax] && loc >= 0 && loc < a.B;
                w += k * wstride;
                u += loc * ustride;
                wstride *= a.K[ax];
                ustride *= a.B;
                t *= ok ? a.taper[loc] : 0.f;
            }
            if (!ok) continue;
            num += bufA[w * a.bs + u].x;
            den += t;
        }
        // undo the scaling: the filter is linear in m_in and scales as
        // |m_ref| / |m_blur|
        const float sr = a.scale[0], sb = a.scale[1], si = a.scale[2];
        const float back = sb > 0.f ? (sr / sb) * si : 0.f;
        out[g] = den > 0.f ? (num / den) * back : 0.f;
    }
}

int grid_of(long long n) {
    long long b = (n + NTHREADS - 1) / NTHREADS;
    return (int)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

}  // namespace

void wiener_free(WienerWork* w) {
    if (!w) return;
    if (w->plans) {
        (void)hipfftDestroy(w->fwd);
        (void)hipfftDestroy(w->inv);
    }
    if (w->buf) (void)hipFree(w->buf);
    if (w->taper) (void)hipFree(w->taper);
    if (w->scale) (void)hipFree(w->scale);
    delete w;
}

const char* wiener_apply(WienerWork** work, int ndim, const int n[3], int block, double eps_rel,
                         const float* ref, const float* blur, const float* in, int nimg, float* out,
                         hipStream_t st) {
    if (block < 2 || (block & 1)) return "block must be even and >= 2";
    if (!(eps_rel >= 0.0)) return "eps_rel must be >= 0";
    WienerWork* W = *work;
    const bool same = W && W->ndim == ndim && W->block == block && W->n[0] == n[0] && W->n[1] == n[1] &&
                      W->n[2] == n[2];
    if (!same) {
        wiener_free(W);
        W = new WienerWork();
        *work = W;
        W->ndim = ndim;
        W->block = block;
        for (int a = 0; a < 3; ++a) W->n[a] = n[a];
        const int h = block / 2;
        W->nwin = 1;
        W->bs = 1;
        for (int a = 0; a < ndim; ++a) {
            W->nwin *= (n[a] - 1) / h + 2;
            W->bs *= block;
        }
        if (hipMalloc(&W->buf, 3 * W->nwin * W->bs * sizeof(hipfftComplex)) != hipSuccess) return "out of memory";
        if (hipMalloc(&W->taper, block * sizeof(float)) != hipSuccess) return "out of memory";
        if (hipMalloc(&W->scale, (3 * NPART + 3) * sizeof(float)) != hipSuccess) return "out of memory";
        std::vector<float> t(block);
        for (int u = 0; u < block; ++u) {
            const double s = std::sin(M_PI * (u + 0.5) / block);
            t[u] = (float)(s * s);
        }
        if (hipMemcpy(W->taper, t.data(), block * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
            return "taper upload failed";
        int dims[3] = {block, block, block};
        if (hipfftPlanMany(&W->fwd, ndim, dims, nullptr, 1, (int)W->bs, nullptr, 1, (int)W->bs, HIPFFT_C2C,
                           (int)(3 * W->nwin)) != HIPFFT_SUCCESS)
            return "hipfftPlanMany (forward) failed";
        if (hipfftPlanMany(&W->inv, ndim, dims, nullptr, 1, (int)W->bs, nullptr, 1, (int)W->bs, HIPFFT_C2C,
                           (int)W->nwin) != HIPFFT_SUCCESS) {
            (void)hipfftDestroy(W->fwd);
            return "hipfftPlanMany (inverse) failed";
        }
        W->plans = true;
    }
    if (hipfftSetStream(W->fwd, st) != HIPFFT_SUCCESS || hipfftSetStream(W->inv, st) != HIPFFT_SUCCESS)
        return "hipfftSetStream failed";
    WArgs a;
    for (int ax = 0; ax < 3; ++ax) {
        a.n[ax] = n[ax];
        a.K[ax] = ax < ndim ? (n[ax] - 1) / (block / 2) + 2 : 1;
    }
    a.ndim = ndim;
    a.B = block;
    a.nwin = W->nwin;
    a.bs = W->bs;
    a.N = (long long)n[0] * n[1] * n[2];
    a.taper = W->taper;
    a.scale = W->scale + 3 * NPART;
    for (int k = 0; k < nimg; ++k) {
        const long long off = k * a.N;
        k_w_maxabs<<<dim3(NPART, 3), NTHREADS, 0, st>>>(ref + off, blur + off, in + off, a.N, W->scale);
        k_w_scale<<<1, NTHREADS, 0, st>>>(W->scale);
        if (hipGetLastError() != hipSuccess) return "scale kernels failed";
        k_w_extract<<<grid_of(3 * a.nwin * a.bs), NTHREADS, 0, st>>>(a, ref + off, blur + off, in + off, W->buf);
        if (hipGetLastError() != hipSuccess) return "extract kernel failed";
        if (hipfftExecC2C(W->fwd, W->buf, W->buf, HIPFFT_FORWARD) != HIPFFT_SUCCESS) return "forward FFT failed";
        k_w_filter<<<(int)a.nwin, NTHREADS, 0, st>>>(a, eps_rel, W->buf);
        if (hipGetLastError() != hipSuccess) return "filter kernel failed";
        if (hipfftExecC2C(W->inv, W->buf, W->buf, HIPFFT_BACKWARD) != HIPFFT_SUCCESS) return "inverse FFT failed";
        k_w_merge<<<grid_of(a.N), NTHREADS, 0, st>>>(a, W->buf, out + off);
        if (hipGetLastError() != hipSuccess) return "merge kernel failed";
    }
    return nullptr;
}

}  // namespace lsrtm
