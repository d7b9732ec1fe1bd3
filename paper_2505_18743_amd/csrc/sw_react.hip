// Linear reactions coupling tracers: the source h phi_k(c_1, ..., c_M) of
// eq:shw with phi_k = sum_j B_kj c_j, taken explicitly in every stage as
// eq:imex_shw takes the reactions.  After the residuals of a stage, each
// tracer's R gets sum_j B_kj int h c_j psi_i, the integrals on the volume
// rule (the sample rule, or Table 1's Gauss-Legendre rule) with the plain
// depth h = max(zeta + z_b, 0) of that stage's state.
//
// P lanes per cell (the power of two >= the rule's n nodes per direction),
// lane b owning the node row y_b, as in the element kernels: the lane forms
// w_a w_b h at its row's nodes once (registers), then for one tracer at a
// time the row's values c_j(x_a, y_b) from the y-interpolated coefficients,
// the products with w h and their x-projections; the y-projections are sums
// over the cell's lanes.  The depth samples are read once for all tracers.
#include "sw_dev.h"

namespace swk {

namespace {

template <int R, int P>
__global__ __launch_bounds__(kWave) void k_react(ReactArgs A) {
  constexpr int N1 = R + 1, NP = N1 * N1, CPB = kWave / P;
  const int lane = threadIdx.x % P, lc = threadIdx.x / P;
  const int cl = blockIdx.x * CPB + lc;
  const bool cv = cl < A.ncell;
  const int clc = cv ? cl : 0;   // in range for every lane
  const int cell = A.cell0 + clc, n = A.n, M = A.M;
  const bool row = lane < n;
  const int b = row ? lane : 0;
  __shared__ double s_z[CPB][NP], s_c[CPB][kMaxReact][NP], s_S[CPB][kMaxReact][NP];
  for (int t = lane; t < (M + 1) * NP; t += P) {
    const int j = t / NP, i = t % NP;
    if (j < M) s_c[lc][j][i] = A.c[j][(size_t)cell * NP + i];
    else s_z[lc][i] = A.z[(size_t)cell * NP + i];
  }
  __syncthreads();
  const double dx = A.cdx[cell], dx2 = dx * dx;
  double lb[N1];
#pragma unroll
  for (int k = 0; k < N1; ++k) lb[k] = A.l[b * N1 + k];
  const double wb = row ? A.w[b] : 0.0;   // rows past n weigh nothing
  // w_a w_b h at the row's nodes (x_a, y_b); depth samples at [a][b]
  double rz[N1];
#pragma unroll
  for (int kx = 0; kx < N1; ++kx) {
    double v = 0.0;
#pragma unroll
    for (int ky = 0; ky < N1; ++ky) v += lb[ky] * s_z[lc][ky * N1 + kx];
    rz[kx] = v;
  }
  const double* zb = A.zb + (size_t)clc * n * n + b;
  double wh[P];
#pragma unroll
  for (int a = 0; a < P; ++a) {
    wh[a] = 0.0;
    if (a < n) {
      double z = 0.0;
#pragma unroll
      for (int kx = 0; kx < N1; ++kx) z += A.l[a * N1 + kx] * rz[kx];
      const double s = z + zb[(size_t)a * n];
      wh[a] = A.w[a] * wb * (s > 0.0 ? s : 0.0);
    }
  }
  for (int j = 0; j < M; ++j) {
    double rc[N1], pr[N1];
#pragma unroll
    for (int kx = 0; kx < N1; ++kx) {
      double v = 0.0;
#pragma unroll
      for (int ky = 0; ky < N1; ++ky) v += lb[ky] * s_c[lc][j][ky * N1 + kx];
      rc[kx] = v;
      pr[kx] = 0.0;
    }
#pragma unroll
    for (int a = 0; a < P; ++a) {
      if (a < n) {
        double la[N1];
#pragma unroll
        for (int k = 0; k < N1; ++k) la[k] = A.l[a * N1 + k];
        double c = 0.0;
#pragma unroll
        for (int kx = 0; kx < N1; ++kx) c += la[kx] * rc[kx];
        const double v = wh[a] * c;
#pragma unroll
        for (int ix = 0; ix < N1; ++ix) pr[ix] += la[ix] * v;
      }
    }
#pragma unroll
    for (int iy = 0; iy < N1; ++iy)
#pragma unroll
      for (int ix = 0; ix < N1; ++ix) {
        const double S = gsum<P>(lb[iy] * pr[ix]);
        if (lane == 0) s_S[lc][j][iy * N1 + ix] = S * dx2;
      }
  }
  __syncthreads();
  // R_k,i += sum_j B_kj S_j,i
  if (!cv) return;
  for (int t = lane; t < M * NP; t += P) {
    const int k = t / NP, i = t % NP;
    double add = 0.0;
    for (int j = 0; j < M; ++j) add += A.B[k * M + j] * s_S[lc][j][i];
    A.res[k][(size_t)cell * NP + i] += add;
  }
}

template <int R>
hipError_t react_r(const ReactArgs& a, hipStream_t s) {
  const int P = lanes_for(a.n), cpb = kWave / P;
  const unsigned nblk = (unsigned)((a.ncell + cpb - 1) / cpb);
  switch (P) {
    case 4: hipLaunchKernelGGL((k_react<R, 4>), dim3(nblk), dim3(kWave), 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_react<R, 8>), dim3(nblk), dim3(kWave), 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_react<R, 16>), dim3(nblk), dim3(kWave), 0, s, a); break;
    case 32: hipLaunchKernelGGL((k_react<R, 32>), dim3(nblk), dim3(kWave), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_react(int r, const ReactArgs& a, hipStream_t s) {
  if (a.ncell <= 0 || a.M <= 0) return hipSuccess;
  if (a.M > kMaxReact || a.n < 1 || a.n > kReactMaxRule || a.N1 != r + 1) return hipErrorInvalidValue;
  switch (r) {
    case 1: return react_r<1>(a, s);
    case 2: return react_r<2>(a, s);
    case 3: return react_r<3>(a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace swk
