// Colour likelihood of the t-links (Section 4: psi_1 = -log p(C | A) with p(C | A) a
// Gaussian mixture over RGB fitted by EM; Section 5: every pixel is a sample, weighted by
// the prior p(A = 1) for the object and by 1 - p for the background; Section 8.1: M = 3).
//
// Per label and iteration: one pass over the pixels accumulates, for every component,
// the responsibility-weighted count, first and second moments about the component's
// current mean (FP32 per pixel, FP64 from the wavefront sum on, one partial per
// workgroup); one workgroup then reduces the partials in a fixed order and computes the
// new weights, means and covariances, their inverses and log-normalisers in FP64.  The
// start is the weighted mean and covariance of each label's samples with the means
// spread along the covariance's leading eigenvector.  A final pass adds psi_1 of both
// labels to the unary costs.  The pixel passes read 7 bytes per pixel.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include <algorithm>

#include "sp_internal.h"
#include "sp_kernels.h"
#include "sp_device.h"

namespace {

constexpr int GPX = SP_GMM_TILE / SP_BLOCK;   // pixels per thread of an accumulation tile
constexpr float kInv255 = 1.f / 255.f;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
constexpr double kLog2Pi = 1.8378770664093453;

__device__ __forceinline__ float ex(float x) { return __builtin_amdgcn_exp2f(x * kLog2e); }
__device__ __forceinline__ float lg(float x) { return __builtin_amdgcn_logf(x) * kLn2; }

// Squared Mahalanobis distance d' P d with P stored as (xx, xy, xz, yy, yz, zz).
__device__ __forceinline__ float quad(const float* P, float dx, float dy, float dz) {
  const float a = P[0] * dx * dx + P[3] * dy * dy + P[5] * dz * dz;
  const float b = P[1] * dx * dy + P[2] * dx * dz + P[4] * dy * dz;
  return fmaf(2.f, b, a);
}

// Moments of one sample with weight wr about the centre: count, first (3) and second (6).
__device__ __forceinline__ void add_moments(float* a, float wr, float dx, float dy, float dz) {
  a[0] += wr;
  const float ux = wr * dx, uy = wr * dy, uz = wr * dz;
  a[1] += ux;
  a[2] += uy;
  a[3] += uz;
  a[4] = fmaf(ux, dx, a[4]);
  a[5] = fmaf(ux, dy, a[5]);
  a[6] = fmaf(ux, dz, a[6]);
  a[7] = fmaf(uy, dy, a[7]);
  a[8] = fmaf(uy, dz, a[8]);
  a[9] = fmaf(uz, dz, a[9]);
}

// EM = false: the start's moments of both labels about (0.5, 0.5, 0.5); EM = true: the
// E-step under the current mixtures and the moments of every component about its mean.
template <int M, bool EM>
__global__ __launch_bounds__(SP_BLOCK) void k_gmm_acc(GmmIO io) {
  constexpr int NC = EM ? M : 1;
  constexpr int NV = 2 * NC * 10;
  __shared__ double red[4][NV];
  const GmmState* st = io.st;
  float acc[2][NC][10];
#pragma unroll
  for (int L = 0; L < 2; ++L)
#pragma unroll
    for (int m = 0; m < NC; ++m)
#pragma unroll
      for (int v = 0; v < 10; ++v) acc[L][m][v] = 0.f;
  const gp<const uint8_t> rgb = G(io.rgb);
  const gp<const float> prior = G(io.prior);
  const uint32_t base = blockIdx.x * SP_GMM_TILE;
#pragma unroll
  for (int k = 0; k < GPX; ++k) {
    const uint32_t i = base + k * SP_BLOCK + threadIdx.x;
    if (i >= (uint32_t)io.n) continue;
    const float cx = (float)rgb[3 * i] * kInv255, cy = (float)rgb[3 * i + 1] * kInv255,
                cz = (float)rgb[3 * i + 2] * kInv255;
    const float pi = prior[i];
    const float w[2] = {1.f - pi, pi};
#pragma unroll
    for (int L = 0; L < 2; ++L) {
      if (!EM) {
        add_moments(acc[L][0], w[L], cx - 0.5f, cy - 0.5f, cz - 0.5f);
        continue;
      }
      if (!st->label_on[L]) continue;
      float lp[NC], mx = -INFINITY;
#pragma unroll
      for (int m = 0; m < NC; ++m) {
        const GmmComp& g = st->comp[L][m];
        lp[m] = g.on ? g.lnorm - 0.5f * quad(g.P, cx - g.mu[0], cy - g.mu[1], cz - g.mu[2]) : -INFINITY;
        mx = fmaxf(mx, lp[m]);
      }
      float r[NC], sum = 0.f;
#pragma unroll
      for (int m = 0; m < NC; ++m) {
        r[m] = st->comp[L][m].on ? ex(lp[m] - mx) : 0.f;
        sum += r[m];
      }
      const float ws = w[L] / sum;
#pragma unroll
      for (int m = 0; m < NC; ++m) {
        const GmmComp& g = st->comp[L][m];
        if (g.on) add_moments(acc[L][m], ws * r[m], cx - g.mu[0], cy - g.mu[1], cz - g.mu[2]);
      }
    }
  }
  const int lane = lane_id(), wv = wave_id();
#pragma unroll
  for (int L = 0; L < 2; ++L)
#pragma unroll
    for (int m = 0; m < NC; ++m)
#pragma unroll
      for (int v = 0; v < 10; ++v) {
        const double s = wave_sum_d((double)acc[L][m][v]);
        if (lane == 0) red[wv][(L * NC + m) * 10 + v] = s;
      }
  __syncthreads();
  for (int v = threadIdx.x; v < NV; v += SP_BLOCK)
    io.part[(size_t)v * io.ntiles + blockIdx.x] = (red[0][v] + red[1][v]) + (red[2][v] + red[3][v]);
}

// Symmetric 3x3 (xx, xy, xz, yy, yz, zz): determinant and inverse by cofactors.
__device__ double sym_inverse(const double* A, double* I) {
  const double c00 = A[3] * A[5] - A[4] * A[4], c01 = A[2] * A[4] - A[1] * A[5], c02 = A[1] * A[4] - A[2] * A[3];
  const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  const double id = 1.0 / det;
  I[0] = c00 * id;
  I[1] = c01 * id;
  I[2] = c02 * id;
  I[3] = (A[0] * A[5] - A[2] * A[2]) * id;
  I[4] = (A[1] * A[2] - A[0] * A[4]) * id;
  I[5] = (A[0] * A[3] - A[1] * A[1]) * id;
  return det;
}

// Positive definite by its leading principal minors.
__device__ bool sym_pd(const double* A) {
  const double m2 = A[0] * A[3] - A[1] * A[1];
  const double det = A[0] * (A[3] * A[5] - A[4] * A[4]) - A[1] * (A[1] * A[5] - A[4] * A[2]) +
                     A[2] * (A[1] * A[4] - A[3] * A[2]);
  return A[0] > 0.0 && m2 > 0.0 && det > 0.0 && isfinite(det);
}

__device__ void set_comp(GmmState* st, int L, int m, double alpha) {
  GmmComp& g = st->comp[L][m];
  double P[6];
  const double det = sym_inverse(st->cov[L][m], P);
  for (int i = 0; i < 3; ++i) g.mu[i] = (float)st->mu[L][m][i];
  for (int i = 0; i < 6; ++i) g.P[i] = (float)P[i];
  g.lnorm = (float)(log(alpha) - 0.5 * log(det) - 1.5 * kLog2Pi);
  g.on = 1;
}

// One workgroup: the partial moments reduced in a fixed order (lane t sums tiles t, t+64, ...,
// then the wavefront sum), then per label (one thread each) the start or the M-step.
template <int M, bool EM>
__global__ __launch_bounds__(SP_BLOCK) void k_gmm_fit(GmmIO io) {
  constexpr int NC = EM ? M : 1;
  constexpr int NV = 2 * NC * 10;
  __shared__ double sums[NV];
  for (int v = wave_id(); v < NV; v += 4) {
    double s = 0.0;
    for (int t = lane_id(); t < io.ntiles; t += 64) s += io.part[(size_t)v * io.ntiles + t];
    s = wave_sum_d(s);
    if (lane_id() == 0) sums[v] = s;
  }
  __syncthreads();
  GmmState* st = io.st;
  if (threadIdx.x < 2) {
    const int L = threadIdx.x;
    if (!EM) {
      const double* a = sums + L * 10;
      const double W0 = a[0];
      st->label_on[L] = W0 > 1e-12 * (double)io.n ? 1 : 0;
      for (int m = 0; m < M; ++m) {
        st->alpha[L][m] = 0.0;
        st->comp[L][m].on = 0;
      }
      if (st->label_on[L]) {
        const double d[3] = {a[1] / W0, a[2] / W0, a[3] / W0};
        const double S[6] = {a[4] / W0 - d[0] * d[0], a[5] / W0 - d[0] * d[1], a[6] / W0 - d[0] * d[2],
                             a[7] / W0 - d[1] * d[1], a[8] / W0 - d[1] * d[2], a[9] / W0 - d[2] * d[2]};
        // leading eigenvector: 64 power steps from (1, 1, 1) / sqrt 3
        double v[3] = {0.5773502691896258, 0.5773502691896258, 0.5773502691896258};
        for (int it = 0; it < 64; ++it) {
          const double u0 = S[0] * v[0] + S[1] * v[1] + S[2] * v[2];
          const double u1 = S[1] * v[0] + S[3] * v[1] + S[4] * v[2];
          const double u2 = S[2] * v[0] + S[4] * v[1] + S[5] * v[2];
          const double nn = sqrt(u0 * u0 + u1 * u1 + u2 * u2);
          if (!(nn > 0.0)) break;
          v[0] = u0 / nn;
          v[1] = u1 / nn;
          v[2] = u2 / nn;
        }
        int k = 0;
        for (int i = 1; i < 3; ++i)
          if (fabs(v[i]) > fabs(v[k])) k = i;
        if (v[k] < 0) v[0] = -v[0], v[1] = -v[1], v[2] = -v[2];
        const double Sv0 = S[0] * v[0] + S[1] * v[1] + S[2] * v[2];
        const double Sv1 = S[1] * v[0] + S[3] * v[1] + S[4] * v[2];
        const double Sv2 = S[2] * v[0] + S[4] * v[1] + S[5] * v[2];
        const double lam = v[0] * Sv0 + v[1] * Sv1 + v[2] * Sv2;
        const double sl = sqrt(fmax(lam, 0.0));
        for (int m = 0; m < M; ++m) {
          const double z = M == 1 ? 0.0 : (m == M - 1 ? 1.0 : m * (2.0 / (M - 1)) - 1.0);
          for (int i = 0; i < 3; ++i) st->mu[L][m][i] = 0.5 + d[i] + z * sl * v[i];
          for (int i = 0; i < 6; ++i) st->cov[L][m][i] = S[i] + ((i == 0 || i == 3 || i == 5) ? (double)io.reg : 0.0);
          st->alpha[L][m] = 1.0 / M;
        }
        for (int m = 0; m < M; ++m)
          if (sym_pd(st->cov[L][m])) set_comp(st, L, m, st->alpha[L][m]);
          else st->alpha[L][m] = 0.0;
      }
    } else if (st->label_on[L]) {
      double W0 = 0.0;
      for (int m = 0; m < M; ++m) W0 += sums[(L * NC + m) * 10];
      double nm[M];
      for (int m = 0; m < M; ++m) {
        const double* a = sums + (L * NC + m) * 10;
        const double N = a[0];
        nm[m] = 0.0;
        if (!st->comp[L][m].on || !(N > 1e-12 * W0)) continue;
        const GmmComp& g = st->comp[L][m];
        const double d[3] = {a[1] / N, a[2] / N, a[3] / N};
        double C[6] = {a[4] / N - d[0] * d[0], a[5] / N - d[0] * d[1], a[6] / N - d[0] * d[2],
                       a[7] / N - d[1] * d[1], a[8] / N - d[1] * d[2], a[9] / N - d[2] * d[2]};
        C[0] += io.reg;
        C[3] += io.reg;
        C[5] += io.reg;
        if (!sym_pd(C)) continue;
        for (int i = 0; i < 3; ++i) st->mu[L][m][i] = (double)g.mu[i] + d[i];
        for (int i = 0; i < 6; ++i) st->cov[L][m][i] = C[i];
        nm[m] = N;
      }
      double tot = 0.0;
      for (int m = 0; m < M; ++m) tot += nm[m];
      for (int m = 0; m < M; ++m) {
        st->alpha[L][m] = tot > 0 ? nm[m] / tot : 0.0;
        if (st->alpha[L][m] > 0.0) set_comp(st, L, m, st->alpha[L][m]);
        else st->comp[L][m].on = 0;
      }
    }
    if (io.out) {
      float* o = io.out + (size_t)L * M * 10;
      for (int m = 0; m < M; ++m) {
        const bool live = st->label_on[L] && st->alpha[L][m] > 0.0;
        o[m * 10] = live ? (float)st->alpha[L][m] : 0.f;
        for (int i = 0; i < 3; ++i) o[m * 10 + 1 + i] = live ? (float)st->mu[L][m][i] : 0.f;
        for (int i = 0; i < 6; ++i) o[m * 10 + 4 + i] = live ? (float)st->cov[L][m][i] : 0.f;
      }
    }
  }
}

// psi_1 = -log sum_m alpha_m N(c; mu_m, Sigma_m), added to the unary cost of its label.
template <int M>
__global__ __launch_bounds__(SP_BLOCK) void k_gmm_psi(GmmIO io) {
  const GmmState* st = io.st;
  const gp<const uint8_t> rgb = G(io.rgb);
  const gp<float> un = G(io.unary);
  for (uint32_t i = blockIdx.x * SP_BLOCK + threadIdx.x; i < (uint32_t)io.n; i += gridDim.x * SP_BLOCK) {
    const float cx = (float)rgb[3 * i] * kInv255, cy = (float)rgb[3 * i + 1] * kInv255,
                cz = (float)rgb[3 * i + 2] * kInv255;
#pragma unroll
    for (int L = 0; L < 2; ++L) {
      if (!st->label_on[L]) continue;
      float lp[M], mx = -INFINITY;
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const GmmComp& g = st->comp[L][m];
        lp[m] = g.on ? g.lnorm - 0.5f * quad(g.P, cx - g.mu[0], cy - g.mu[1], cz - g.mu[2]) : -INFINITY;
        mx = fmaxf(mx, lp[m]);
      }
      if (!(mx > -INFINITY)) continue;
      float sum = 0.f;
#pragma unroll
      for (int m = 0; m < M; ++m) sum += st->comp[L][m].on ? ex(lp[m] - mx) : 0.f;
      const uint32_t o = (uint32_t)L * (uint32_t)io.n + i;
      un[o] = un[o] - (mx + lg(sum));
    }
  }
}

template <int M>
hipError_t launch_m(int phase, const GmmIO& io, hipStream_t st) {
  switch (phase) {
    case 0: hipLaunchKernelGGL((k_gmm_acc<M, false>), dim3(io.ntiles), dim3(SP_BLOCK), 0, st, io); break;
    case 1: hipLaunchKernelGGL((k_gmm_fit<M, false>), dim3(1), dim3(SP_BLOCK), 0, st, io); break;
    case 2: hipLaunchKernelGGL((k_gmm_acc<M, true>), dim3(io.ntiles), dim3(SP_BLOCK), 0, st, io); break;
    case 3: hipLaunchKernelGGL((k_gmm_fit<M, true>), dim3(1), dim3(SP_BLOCK), 0, st, io); break;
    default: {
      const int blocks = (int)std::min<long long>(((long long)io.n + SP_BLOCK - 1) / SP_BLOCK, 4096);
      hipLaunchKernelGGL(k_gmm_psi<M>, dim3(blocks), dim3(SP_BLOCK), 0, st, io);
    }
  }
  return hipGetLastError();
}

}  // namespace

hipError_t sp_launch_gmm(int phase, int M, const GmmIO& io, hipStream_t st) {
  if (io.n <= 0) return hipSuccess;
  switch (M) {
    case 1: return launch_m<1>(phase, io, st);
    case 2: return launch_m<2>(phase, io, st);
    case 3: return launch_m<3>(phase, io, st);
    case 4: return launch_m<4>(phase, io, st);
    default: return hipErrorInvalidValue;
  }
}
