// Attribute baking (Sec. 4 "Inference": covariances and opacities are baked
// into the primitives) and its adjoint for fitting.
//   Sigma = M M^T, M = R(q/|q|) diag(exp(logscale)),  opacity = sigmoid(logit)
// One thread per Gaussian, structure-of-arrays planes, HBM-bound.
#include "vrs_common.h"

namespace vrs {

__device__ inline void quat_rot(float w, float x, float y, float z, float R[3][3]) {
  R[0][0] = 1.0f - 2.0f * (y * y + z * z);
  R[0][1] = 2.0f * (x * y - w * z);
  R[0][2] = 2.0f * (x * z + w * y);
  R[1][0] = 2.0f * (x * y + w * z);
  R[1][1] = 1.0f - 2.0f * (x * x + z * z);
  R[1][2] = 2.0f * (y * z - w * x);
  R[2][0] = 2.0f * (x * z - w * y);
  R[2][1] = 2.0f * (y * z + w * x);
  R[2][2] = 1.0f - 2.0f * (x * x + y * y);
}

__global__ __launch_bounds__(256) void k_bake(const float* __restrict__ ls,
                                              const float* __restrict__ q,
                                              const float* __restrict__ logit, int64_t n,
                                              float* __restrict__ cov, float* __restrict__ op) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  float w = q[i], x = q[n + i], y = q[2 * n + i], z = q[3 * n + i];
  const float inv = rsqrtf(w * w + x * x + y * y + z * z);
  w *= inv; x *= inv; y *= inv; z *= inv;
  float R[3][3];
  quat_rot(w, x, y, z, R);
  float s2[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) s2[k] = __expf(2.0f * ls[k * n + i]);
  float S[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) {
      float acc = 0.0f;
#pragma unroll
      for (int k = 0; k < 3; ++k) acc += R[a][k] * s2[k] * R[b][k];
      S[a][b] = acc;
    }
  cov[i] = S[0][0];
  cov[n + i] = S[0][1];
  cov[2 * n + i] = S[0][2];
  cov[3 * n + i] = S[1][1];
  cov[4 * n + i] = S[1][2];
  cov[5 * n + i] = S[2][2];
  op[i] = 1.0f / (1.0f + __expf(-logit[i]));
}

// Adjoint.  With G the symmetric matrix of dL/dSigma (off-diagonal entries of
// the 6-vector gradient split in half), dL/dM = 2 G M, dL/ds_k =
// sum_i R_ik (dL/dM)_ik, dL/dR_ik = (dL/dM)_ik s_k, then through the
// quaternion's rotation matrix and its normalisation.
__global__ __launch_bounds__(256) void k_bake_bwd(
    const float* __restrict__ ls, const float* __restrict__ q, const float* __restrict__ logit,
    int64_t n, const float* __restrict__ dcov, const float* __restrict__ dop,
    float* __restrict__ dls, float* __restrict__ dq, float* __restrict__ dlogit) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float qw = q[i], qx = q[n + i], qy = q[2 * n + i], qz = q[3 * n + i];
  const float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  const float w = qw / qn, x = qx / qn, y = qy / qn, z = qz / qn;
  float R[3][3];
  quat_rot(w, x, y, z, R);
  float s[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) s[k] = __expf(ls[k * n + i]);
  float G[3][3];
  G[0][0] = dcov[i];
  G[1][1] = dcov[3 * n + i];
  G[2][2] = dcov[5 * n + i];
  G[0][1] = G[1][0] = 0.5f * dcov[n + i];
  G[0][2] = G[2][0] = 0.5f * dcov[2 * n + i];
  G[1][2] = G[2][1] = 0.5f * dcov[4 * n + i];
  float dM[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float acc = 0.0f;
#pragma unroll
      for (int b = 0; b < 3; ++b) acc += G[a][b] * R[b][k] * s[k];
      dM[a][k] = 2.0f * acc;
    }
  float dR[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float ds = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      ds += R[a][k] * dM[a][k];
      dR[a][k] = dM[a][k] * s[k];
    }
    dls[k * n + i] += ds * s[k];
  }
  // dR/d(w,x,y,z) of the rotation matrix of a unit quaternion
  const float gw = 2.0f * (-z * dR[0][1] + y * dR[0][2] + z * dR[1][0] - x * dR[1][2] -
                           y * dR[2][0] + x * dR[2][1]);
  const float gx = 2.0f * (y * dR[0][1] + z * dR[0][2] + y * dR[1][0] - 2.0f * x * dR[1][1] -
                           w * dR[1][2] + z * dR[2][0] + w * dR[2][1] - 2.0f * x * dR[2][2]);
  const float gy = 2.0f * (-2.0f * y * dR[0][0] + x * dR[0][1] + w * dR[0][2] + x * dR[1][0] +
                           z * dR[1][2] - w * dR[2][0] + z * dR[2][1] - 2.0f * y * dR[2][2]);
  const float gz = 2.0f * (-2.0f * z * dR[0][0] - w * dR[0][1] + x * dR[0][2] + w * dR[1][0] -
                           2.0f * z * dR[1][1] + y * dR[1][2] + x * dR[2][0] + y * dR[2][1]);
  const float dot = gw * w + gx * x + gy * y + gz * z;
  dq[i] += (gw - w * dot) / qn;
  dq[n + i] += (gx - x * dot) / qn;
  dq[2 * n + i] += (gy - y * dot) / qn;
  dq[3 * n + i] += (gz - z * dot) / qn;
  if (dop) {
    const float o = 1.0f / (1.0f + __expf(-logit[i]));
    dlogit[i] += dop[i] * o * (1.0f - o);
  }
}

}  // namespace vrs

using namespace vrs;

extern "C" vrs_status vrs_bake_gaussians(const float* logscale, const float* quat,
                                         const float* logit, int64_t n, float* cov,
                                         float* opacity, void* stream) {
  if (n < 0 || (n > 0 && (!logscale || !quat || !logit || !cov || !opacity))) return VRS_EINVAL;
  if (n == 0) return VRS_OK;
  hipLaunchKernelGGL(k_bake, dim3(div_up(n, 256)), dim3(256), 0, static_cast<hipStream_t>(stream),
                     logscale, quat, logit, n, cov, opacity);
  VRS_LAUNCH_CHECK();
  return VRS_OK;
}

extern "C" vrs_status vrs_bake_gaussians_backward(const float* logscale, const float* quat,
                                                  const float* logit, int64_t n,
                                                  const float* d_cov, const float* d_opacity,
                                                  float* d_logscale, float* d_quat,
                                                  float* d_logit, void* stream) {
  if (n < 0 || (n > 0 && (!logscale || !quat || !logit || !d_cov || !d_logscale || !d_quat)))
    return VRS_EINVAL;
  if (d_opacity && !d_logit) return VRS_EINVAL;
  if (n == 0) return VRS_OK;
  hipLaunchKernelGGL(k_bake_bwd, dim3(div_up(n, 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), logscale, quat, logit, n, d_cov, d_opacity,
                     d_logscale, d_quat, d_logit);
  VRS_LAUNCH_CHECK();
  return VRS_OK;
}
