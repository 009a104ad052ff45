// Launchers of the HIP kernels (implemented in sp_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include "sp_internal.h"

hipError_t sp_launch(int kind, const Job* jobs, int n, const StreamDesc* sds, const StepIO* ios,
                     const StepIO* io0, int flag, const float* aux, hipStream_t st, size_t lds = 0);
hipError_t sp_csapply_reserve_lds(size_t bytes);
hipError_t sp_launch_bwd(int kind, const Job* jobs, int n, const StreamDesc* sds, const BwdIO* bios,
                         const BwdIO* b0, hipStream_t st);
hipError_t sp_launch_consp_dot(const Job* jobs, int n, const StreamDesc* sds, const StepIO* ios,
                               const float* gs_all, const float* ms_all, const int* frame_of,
                               float* dot_part, float* cx_out, hipStream_t st);
hipError_t sp_launch_bwd_final(int T, int n_lvl0_tiles, int n_cmax_tiles, const float* gk_part,
                               const float* dot_part, const float* cx, const float* ms_all, const double* Kd,
                               const double* Pd, double Q, double R, const float* w, float flat_tol,
                               double* gK_scratch, float* grad_w, float* grad_q, float* grad_r, hipStream_t st);
hipError_t sp_launch_loss(const float* prior, const uint8_t* mask, size_t n, float* grad, float* part, int nblk,
                          float* loss, hipStream_t st);
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
