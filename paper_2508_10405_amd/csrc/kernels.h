// Host-side launchers of the device kernels.
#pragma once
#include <hip/hip_runtime.h>
#include "common.h"

namespace lsrtm {

// Stencil phases (see kern2d.hip / kern3d.hip).
enum Kind {
    K_BG_V = 0,    // background velocity phase
    K_BG_P = 1,    // background pressure phase
    K_SEG_V = 2,   // background velocity phase, stores G_a p + psi_a (replay)
    K_SEG_P = 3,   // background pressure phase, stores q (replay)
    K_BORN_V = 4,  // background + scattered velocity phase
    K_BORN_P = 5,  // background + scattered pressure phase
    K_ADJ_A = 6,   // adjoint pressure phase + lnkappa imaging
    K_ADJ_B = 7,   // adjoint velocity phase + lnrho imaging
    K_BORN_V_RC = 8,   // 2D scattered velocity phase on a background read from the replay cache
    K_BORN_P_RC = 9    // 2D scattered pressure phase on a background read from the replay cache
};

extern const int kTiles2[][2];
extern const int kNumTiles2;
extern const int kTiles3[][3];
extern const int kNumTiles3;

hipError_t launch2d(int kind, int tile_id, int ntiles, hipStream_t st, const Slot* slots,
                    const int4* tiles, const Coef& C, int n, int sstep, int flag, const TileRec& tr,
                    hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch3d(int kind, int tile_id, int ntiles, hipStream_t st, const Slot* slots,
                    const int4* tiles, const Coef& C, int n, int sstep, int flag,
                    hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Fused 2D schedule (kern2f.hip): one kernel per step; kind is K_BG_V,
// K_SEG_V, K_BORN_V (whole forward step) or K_ADJ_A (whole adjoint step).
hipError_t launch2f(int kind, int tile_id, int ntiles, hipStream_t st, const Slot* slots,
                    const int4* tiles, const Coef& C, int n, int sstep, int flag, const TileRec& tr,
                    hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Every stencil launcher takes an optional event pair that receives the
// kernel's start and end (timing).

// Auxiliary kernels (aux.hip).
hipError_t launch_fill(float* p, long long n, float v, hipStream_t st);
hipError_t launch_fill_f64(double* p, long long n, hipStream_t st);

// Model on a shot's padded grid from the global physical logs (edge-replicated
// into the PML): kdt = dt*exp(lnvp+lnip); sb = sqrt(dt)*exp(-lnrho/2), so that
// dt*b_a = dt*exp(-(lnrho_i + lnrho_i+1)/2) at the half node i + 1/2 is the
// FP32 product sb_i * sb_i+1.  The kernels form that product from sb (one
// array instead of ndim); bdt_a, when not null, holds the same products for
// the fused 2D adjoint, which reads dt b_a on its velocity halo.
struct PrepArgs {
    const float* lnvp; const float* lnip;   // global physical arrays
    int gn[3];                              // global physical sizes (z, x, y)
    int lo[3], wn[3];                       // window origin and size
    int npml;
    int N[3];                               // padded sizes
    long long sx, sy;                       // strides
    double dt;
    int ndim;
    float* kdt; float* sb; float* bdt[3];
};
hipError_t launch_model_prep(const PrepArgs& a, hipStream_t st);

// Perturbation on a shot's padded grid: dlnr = dlnIp - dlnVp,
// dlnk = dlnIp + dlnVp inside the window, zero in the PML.
struct DmArgs {
    const float* dm;                        // [2][gpts] global (dlnVp, dlnIp)
    long long gpts;
    int gn[3];
    int lo[3], wn[3];
    int npml;
    int N[3];
    long long sx, sy;
    int ndim;
    float* dlnr; float* dlnk;
};
hipError_t launch_dm_prep(const DmArgs& a, hipStream_t st);

// Receivers.
hipError_t launch_gather(const Slot* slots, const Rec* rec, int nrec, int n, int from_scattered,
                         float* d, hipStream_t st);
// Injection of d[it = n] into the adjoint pressure: one thread per distinct
// receiver node, summing its receivers in a fixed order.  The adjoint state
// holds Q = -dt kappa p~, so the sum s enters as -dt kappa s.
hipError_t launch_inject(const Slot* slots, const int* node_slot, const int* node_idx,
                         const int* node_ptr, const Rec* rec, int nnode, int n, const float* d,
                         hipStream_t st);

// Images of a launch group added into the FP64 global accumulator
// acc[2][gpts] (lnVp, lnIp): img_lnVp = -g_lnrho + g_lnkappa,
// img_lnIp = g_lnrho + g_lnkappa, slots taken in order.
struct ImgArgs {
    const Slot* slots;
    const int* win;        // [nslot][6] window lo/hi (z, x, y) of each slot
    int nslot;
    int ndim;
    int gn[3];
    int npml;
    double* acc;
    long long gpts;
};
hipError_t launch_image_reduce(const ImgArgs& a, hipStream_t st);
hipError_t launch_image_store(const double* acc, float* img, long long n, int accumulate,
                              hipStream_t st);
// Pseudo-Hessian: slot sums -> acc[2][gpts] (shot order), then h and the
// diagonal inverse 1 / (h + eps) for both parameters.
hipError_t launch_ph_reduce(const ImgArgs& a, hipStream_t st);
hipError_t launch_ph_finish(const double* acc, const float* lnvp, const float* lnip, double dt, float* h,
                            long long n, hipStream_t st);
hipError_t launch_ph_minv(const float* h, double eps, float* minv, long long n, hipStream_t st);
hipError_t launch_mul(const float* a, const float* b, float* out, long long n, hipStream_t st);

// Top mute of recorded data, in place (aux.hip).
hipError_t launch_mute_tables(const Slot* slots, const Rec* rec, int nrec, int ndim, const double* h, double t0,
                              double v_mute, long long* off, int* stride, double* tc, hipStream_t st);
hipError_t launch_mute(float* d, const long long* off, const int* stride, const double* tc, int nrec, int nt,
                       double dt, int ntaper, hipStream_t st);

// Interpolated PSF Hessian (psf.hip).
struct PsfArgs {
    int n[3];              // physical sizes (z, x, y); n[2] = 1 in 2D
    int ndim;
    int W;                 // window half-width
    int mono;              // 1 = the lnIp block only
    long long N;           // n[0] * n[1] * n[2]
    const int* tab;        // per coordinate of each axis: corner c0, corner c1, weight (float bits)
    int off[3];            // first coordinate of axis a in tab
    const float* psf;      // PSF images [2 (scatterer parameter q)][2 (response p)][N]
};
hipError_t launch_psf_apply(const PsfArgs& a, const float* x, float* y, int transpose, hipStream_t st);
hipError_t launch_psf_spikes(const PsfArgs& a, int q, float* dm, hipStream_t st);

// Nonstationary Wiener deblurring (wiener.hip): FFT plans and buffers kept
// between calls; returns nullptr or an error message.
struct WienerWork;
const char* wiener_apply(WienerWork** work, int ndim, const int n[3], int block, double eps_rel,
                         const float* ref, const float* blur, const float* in, int nimg, float* out,
                         hipStream_t st);
void wiener_free(WienerWork* w);

// Max |x| of a physical float array (finite check: non-finite -> +inf).
hipError_t launch_maxabs(const float* x, long long n, float* partial, int nblk, hipStream_t st);
// Per-block maximum of x (non-finite -> +inf); partial[nblk].
hipError_t launch_maxval(const float* x, long long n, float* partial, int nblk, hipStream_t st);

// FP64 dot product (two stages, fixed order) and FP64-rounded axpy / xpby.
hipError_t launch_dot(const float* a, const float* b, long long n, double* partial, int nblk,
                      double* out, hipStream_t st);
hipError_t launch_axpy(double alpha, const float* x, float* y, long long n, hipStream_t st);
hipError_t launch_xpby(const float* x, double beta, float* y, long long n, hipStream_t st);
hipError_t launch_copy(const float* x, float* y, long long n, hipStream_t st);
// Calibration: one streaming pass over a mix of nread + nwrite arrays of n
// floats in buf, in order (grid = NULL) or in the 3D tiles' order over the
// grid (nz, nx, ny, ldz); (nread, nwrite) one of (10, 6), (10, 2), (5, 6),
// (5, 2), (2, 1), else hipErrorInvalidValue.
hipError_t launch_stream_mix(float* buf, long long n, int nread, int nwrite, const int* grid, hipStream_t st,
                             hipEvent_t e0, hipEvent_t e1);

// Checkpoints: per slot, fields p, v_a as FP32/FP16/BF16 with a max-abs scale
// per field, CPML memories of the strips as FP32.
struct CkptArgs {
    const Slot* slots;
    int nslot;
    int ndim;
    int dtype;                     // 0 f32, 1 f16, 2 bf16
    int S;                         // strip depth per side
    int j;                         // checkpoint index >= 1 (Slot::ck + (j-1) * Slot::ckbytes)
    float* scales;                 // [nslot][1+ndim] scales of checkpoint j
    float* partial;                // reduction workspace [nslot][1+ndim][nblk]
    int nblk;
    int* nonfinite;                // set to 1 if a field holds NaN/Inf
};
hipError_t launch_ckpt_save(const CkptArgs& a, long long max_npts, hipStream_t st);
hipError_t launch_ckpt_load(const CkptArgs& a, long long max_npts, hipStream_t st);

}  // namespace lsrtm
