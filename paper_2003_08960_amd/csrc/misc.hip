// Envelope cuts (text after Eq. 7: three orthogonal cuts of the magnitude of
// the rendered volume at user-selected positions) and the final FP64
// reduction of the sharpness gradient.
#include "internal.hpp"

namespace ssoct {

// One thread per output value: N*N (xy) + T*N (xz) + T*N (yz).
__global__ void k_cuts(int T, int N, const float2* __restrict__ vol, int x0, int y0, int q0, int power,
                       float* __restrict__ cut_xy, float* __restrict__ cut_xz, float* __restrict__ cut_yz) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nxy = (size_t)N * N, nz = (size_t)T * N;
  size_t src;
  float* dst;
  if (i < nxy) {
    src = (size_t)q0 * nxy + i;
    dst = cut_xy + i;
  } else if (i < nxy + nz) {
    const size_t k = i - nxy, q = k / N, v = k % N;
    src = q * nxy + (size_t)y0 * N + v;
    dst = cut_xz + k;
  } else if (i < nxy + 2 * nz) {
    const size_t k = i - nxy - nz, q = k / N, u = k % N;
    src = q * nxy + u * N + x0;
    dst = cut_yz + k;
  } else {
    return;
  }
  const float2 v = vol[src];
  const float m2 = v.x * v.x + v.y * v.y;
  *dst = power ? m2 : sqrtf(m2);
}

hipError_t launch_cuts(int T, int N, const float2* vol, int x0, int y0, int q0, int power, float* cut_xy,
                       float* cut_xz, float* cut_yz, hipStream_t s) {
  const size_t n = (size_t)N * N + 2 * (size_t)T * N;
  const int block = 256;
  hipLaunchKernelGGL(k_cuts, dim3((unsigned)((n + block - 1) / block)), dim3(block), 0, s, T, N, vol, x0, y0, q0,
                     power, cut_xy, cut_xz, cut_yz);
  return hipGetLastError();
}

// Single workgroup of GF_THREADS.  mono_partials[t][nblk][15] are per-block
// moments M_ab = sum Im(conj(g) z) x^a y^b; zmat[j][k] expands Zernike j in
// the monomials.  Gradients (chain of the sharpness loss):
//   dL/dphi_t = -M_00(t),  dL/dz = -sum_t (alpha_t / z) (N^2 / 2) (M_20 + M_02)(t),
//   dL/dc_j   = -sum_t sum_k zmat[j][k] M_k(t),   all times grad_scale.
// Every sum runs in a fixed order (strided per thread, butterfly per wave,
// waves in index order), so the result does not depend on timing.
constexpr int GF_THREADS = 1024;

__global__ __launch_bounds__(GF_THREADS) void k_grad_finish(int T, int N, int nblk,
                                                            const double* __restrict__ mono_partials,
                                                            const double* __restrict__ loss_partials, int n_loss,
                                                            const double* __restrict__ alpha_over_z,
                                                            const double* __restrict__ zmat, double grad_scale,
                                                            double* __restrict__ out) {
  constexpr int NWV = GF_THREADS / 64;
  __shared__ double red[NWV][N_MONO + 2];
  __shared__ double zs[15 * N_MONO];
  const int tid = threadIdx.x;
  if (tid < 15 * N_MONO) zs[tid] = zmat[tid];   // in flight while the partials are summed
  const double half_n2 = 0.5 * (double)N * (double)N;
  for (int t = tid; t < T; t += GF_THREADS) {
    double m0 = 0.0;
#pragma unroll 8
    for (int b = 0; b < nblk; ++b) m0 += mono_partials[((size_t)t * nblk + b) * N_MONO];
    out[1 + 1 + 15 + t] = -grad_scale * m0;
  }
  double acc[N_MONO + 2];
#pragma unroll
  for (int k = 0; k < N_MONO + 2; ++k) acc[k] = 0.0;
  const int rows = T * nblk;
#pragma unroll 2
  for (int i = tid; i < rows; i += GF_THREADS) {
    const double* p = mono_partials + (size_t)i * N_MONO;
    const double w = alpha_over_z[i / nblk] * half_n2;
#pragma unroll
    for (int k = 0; k < N_MONO; ++k) acc[k] += p[k];
    acc[N_MONO] += w * (p[3] + p[5]);
  }
#pragma unroll 8
  for (int i = tid; i < n_loss; i += GF_THREADS) acc[N_MONO + 1] += loss_partials[i];
#pragma unroll
  for (int k = 0; k < N_MONO + 2; ++k) {
    double a = acc[k];
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    acc[k] = a;
  }
  if ((tid & 63) == 0) {
#pragma unroll
    for (int k = 0; k < N_MONO + 2; ++k) red[tid >> 6][k] = acc[k];
  }
  __syncthreads();
  if (tid < N_MONO + 2) {
    double s = 0.0;
    for (int w = 0; w < NWV; ++w) s += red[w][tid];
    red[0][tid] = s;
  }
  __syncthreads();
  const double* M = red[0];
  if (tid < 15) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < N_MONO; ++k) s += zs[tid * N_MONO + k] * M[k];
    out[2 + tid] = -grad_scale * s;
  } else if (tid == 15) {
    out[0] = M[N_MONO + 1];
    out[1] = -grad_scale * M[N_MONO];
  }
}

hipError_t launch_grad_finish(int T, int N, int nblk, const double* mono_partials, const double* loss_partials,
                              int n_loss, const double* alpha_over_z, const double* zmat, double grad_scale,
                              double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_finish, dim3(1), dim3(GF_THREADS), 0, s, T, N, nblk, mono_partials, loss_partials, n_loss,
                     alpha_over_z, zmat, grad_scale, out);
  return hipGetLastError();
}

}  // namespace ssoct
