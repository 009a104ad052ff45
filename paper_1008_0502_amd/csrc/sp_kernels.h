// Launchers of the HIP kernels (implemented in sp_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include "sp_internal.h"

hipError_t sp_launch(int kind, const Job* jobs, int n, const StreamDesc* sds, const StepIO* ios,
                     const StepIO* io0, int flag, const float* aux, hipStream_t st, size_t lds = 0);
hipError_t sp_csapply_reserve_lds(size_t bytes);
hipError_t sp_launch_bwd(int kind, const Job* jobs, int n, const StreamDesc* sds, const BwdIO* bios,
                         const BwdIO* b0, hipStream_t st);
// Conspicuity recomputed from checkpoints, dotted with each frame's saliency adjoint
// (per-frame buffers named by ios[stream]: gs, dot, cx, ms_tape).
hipError_t sp_launch_consp_dot(const Job* jobs, int n, const StreamDesc* sds, const StepIO* ios, hipStream_t st);
// Adjoint reduction: one workgroup per stream of tab (or the single stream *one when tab
// is null), shared gains Kd and variances Pd of T steps.
hipError_t sp_launch_bwd_final(const BwdFin* tab, const BwdFin* one, int n_streams, int T, const double* Kd,
                               const double* Pd, double Q, double R, float flat_tol, hipStream_t st);
// Masked-MSE loss of n_streams clips (tab) or of the single clip *one, nblk partials each.
hipError_t sp_launch_loss(const LossIO* tab, const LossIO* one, int n_streams, int nblk, hipStream_t st);
// The colour-statistics launch of a batched step, which also starts the step (see
// BatchBegin).  RgbNodeArgs holds the argument values of that launch as a graph kernel
// node; sp_batch_rgb_node_params points p at them so the node can be re-pointed at the
// next step's frame table (the values must outlive the update call).
hipError_t sp_launch_batch_rgb(const Job* jobs, int n_jobs, const StreamDesc* sds, StepIO* ios, int want_d2,
                               const BatchBegin& bb, hipStream_t stream);
struct RgbNodeArgs {
  const Job* jobs;
  const StreamDesc* sds;
  const StepIO* ios;
  StepIO io0;
  int want_d2;
  BatchBegin bb;
  void* argv[6];
};
void sp_batch_rgb_node_params(RgbNodeArgs* a, int n_jobs, hipKernelNodeParams* p);
hipError_t sp_launch_batch_reset(int n, BatchState* st, hipStream_t stream);
hipError_t sp_launch_batch_copy_out(int n, const BatchState* st, const StreamDesc* sds, float* const* out,
                                    hipStream_t stream);
// Counter calibration copy of n16 16-byte units (mode: 0 dword, 1 dwordx4, 2 global->LDS dword).
hipError_t sp_launch_calib(const float* src, float* dst, size_t n16, int mode, hipStream_t st);

// Device address of the allocation-free entry point's scratch array on the current device
// (SP_NOALLOC_BYTES bytes; looked up once per device, then remembered).
hipError_t sp_noalloc_scratch(void** ptr);
// Prior of the first frame from manual labels (n pixels).
hipError_t sp_launch_manual(const uint8_t* labels, float* pnext, float* pout, size_t n, float eps, hipStream_t st);
// Colour likelihood phases: 0 start moments, 1 start fit, 2 E-step moments, 3 M-step fit,
// 4 psi added to the unary costs (M = components per label, 1..SP_GMM_MAXM).
hipError_t sp_launch_gmm(int phase, int M, const GmmIO& io, hipStream_t st);
// Minimum cut phases: 0 counters + capacities, 1 relabel pass (flags cleared first),
// 2 push / relabel cycles, 3 labels and the flow value.
hipError_t sp_launch_cut(int phase, const CutIO& io, hipStream_t st);
// Pixel-level adjoint passes (sp_pixadj.hip).  sp_pa_plane kinds: 0 pyramid-step transpose
// (flag: accumulate), 1 centre-surround map, 2 centre-surround adjoint (adds to gc[plane]),
// 3 up-sample transpose (subtracts).  sp_pa_gabor: the Gabor transposes of every level in
// L (taps: [4][2 SP_PA_R + 1]^2, radius = plane d), max_tiles the most 16x16 tiles of a level.
hipError_t sp_pa_gs(const float* gs, const float* S, const float* ms, int n, float flat_tol, float* gS,
                    double* part, hipStream_t st);   // part: (n + 255) / 256 doubles of scratch
hipError_t sp_pa_nadjoint(const PaMap* maps, int nmaps, int maxn, int maxh, float flat_tol, hipStream_t st);
hipError_t sp_pa_plane(int kind, const PaPlane* tab, int nplanes, int maxn, int flag, float* const* gc,
                       const float* taps, hipStream_t st, int gabor_r = 0);
hipError_t sp_pa_gabor(const PaGabLevels& L, int max_tiles, const float* taps, hipStream_t st, int gabor_r);
hipError_t sp_pa_feat(const uint8_t* rgb, const uint8_t* prev, const uint32_t* maxp, int nmax, const float* g0, int n,
                      float* gout, float* gprev, hipStream_t st);
hipError_t sp_pa_zero(float* p, size_t n, hipStream_t st);
