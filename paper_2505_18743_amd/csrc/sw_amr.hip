// Kernels of the dynamic h-adaptivity (Sec. 3.3 refinement criteria; Sec. 3.4
// conservative remap, eq:cons-remap, and the mass source Q^n, eq:mass-loss):
// the per-cell refinement indicator, the remap of the state onto the new
// quadtree, bathymetry sampled from a raster at the new cells' nodes, and the
// per-cell mass and bathymetry integrals of the Q^n diagnostic.
#include "sw_dev.h"

namespace swk {

namespace {

constexpr int kAmrLanes = 64;   // one wavefront per cell

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) v = fmax(v, __shfl_xor(v, m));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m);
  return v;
}

// eta_K: one wavefront per cell, lanes over the n x n nodes of the volume
// rule.  Vorticity of u = q / h_des (eq:velocity) by the chain rule with the
// depth gradient grad zeta at wet nodes, or |grad c|.
__global__ __launch_bounds__(kAmrLanes) void k_amr_eta(AmrEtaArgs A) {
  const int cl = blockIdx.x;
  if (cl >= A.ncell) return;
  const int cell = A.cell0 + cl, N1 = A.N1, NP = N1 * N1, n = A.n;
  __shared__ double s[4][16];
  for (int k = threadIdx.x; k < NP; k += blockDim.x) {
    s[0][k] = A.z[(size_t)cell * NP + k];
    s[1][k] = A.qx[(size_t)cell * NP + k];
    s[2][k] = A.qy[(size_t)cell * NP + k];
    s[3][k] = A.c ? A.c[(size_t)cell * NP + k] : 0.0;
  }
  __syncthreads();
  const double idx = 1.0 / A.cdx[cell];
  const double eps = A.eps, e4 = (eps * eps) * (eps * eps);
  double best = 0.0;
  for (int q = threadIdx.x; q < n * n; q += blockDim.x) {
    const int a = q % n, b = q / n;   // node (x_a, y_b)
    double v[4] = {0, 0, 0, 0}, vx[4] = {0, 0, 0, 0}, vy[4] = {0, 0, 0, 0};
    for (int jy = 0; jy < N1; ++jy) {
      const double lb = A.l[b * N1 + jy], db = A.d[b * N1 + jy];
      for (int jx = 0; jx < N1; ++jx) {
        const double la = A.l[a * N1 + jx], da = A.d[a * N1 + jx];
        for (int f = 0; f < 4; ++f) {
          const double u = s[f][jy * N1 + jx];
          v[f] += la * lb * u;
          vx[f] += da * lb * u;
          vy[f] += la * db * u;
        }
      }
    }
    double val;
    if (A.kind == 0) {
      const double sdep = v[0] + A.zb[((size_t)cl * n + a) * n + b];
      const bool wet = sdep > 0.0;
      const double h = wet ? sdep : 0.0;
      const double ih = inv_des(h, eps);
      double dih = 0.0;
      if (h >= eps) {
        dih = -1.0 / (h * h);
      } else if (h > 0.0) {
        const double h4 = (h * h) * (h * h), t = e4 + h4;
        dih = 1.4142135623730951 * (e4 - h4) / (t * sqrt(t));
      }
      const double hx = wet ? vx[0] * idx : 0.0, hy = wet ? vy[0] * idx : 0.0;
      val = fabs(ih * (vx[2] * idx - vy[1] * idx) + dih * (v[2] * hx - v[1] * hy));
    } else {
      const double cx = vx[3] * idx, cy = vy[3] * idx;
      val = sqrt(cx * cx + cy * cy);
    }
    best = fmax(best, val);
  }
  best = wave_max(best);
  if (threadIdx.x == 0) A.eta[cell] = best;
}

// Remap to the new cells, one thread per (new cell, nodal value): a copy, the
// parent's polynomial at the child's support points, or the exact-mass L2
// projection of four children; per-cell scalars (Manning, bed offset) are
// inherited by a child and averaged into a parent.
__global__ void k_amr_transfer(AmrXferArgs A) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int NP = A.NP;
  if (t >= A.Kn * NP) return;
  const int nc = t / NP, j = t % NP;
  const int ty = A.type[nc];
  const int* s = A.src + 4 * (size_t)nc;
  for (int f = 0; f < 4; ++f) {
    if (!A.out[f]) continue;
    const double* in = A.in[f];
    double v = 0.0;
    if (ty == 0) {
      v = in[(size_t)s[0] * NP + j];
    } else if (ty == 1) {
      const double* T = A.tchild + ((size_t)s[1] * NP + j) * NP;
      for (int k = 0; k < NP; ++k) v += T[k] * in[(size_t)s[0] * NP + k];
    } else {
      for (int c = 0; c < 4; ++c) {
        const double* T = A.tproj + ((size_t)c * NP + j) * NP;
        for (int k = 0; k < NP; ++k) v += T[k] * in[(size_t)s[c] * NP + k];
      }
    }
    A.out[f][(size_t)nc * NP + j] = v;
  }
  if (j == 0) {
    if (ty == 2) {
      A.nman_out[nc] = 0.25 * (A.nman_in[s[0]] + A.nman_in[s[1]] + A.nman_in[s[2]] + A.nman_in[s[3]]);
      A.db_out[nc] = 0.25 * (A.db_in[s[0]] + A.db_in[s[1]] + A.db_in[s[2]] + A.db_in[s[3]]);
    } else {
      A.nman_out[nc] = A.nman_in[s[0]];
      A.db_out[nc] = A.db_in[s[0]];
    }
  }
}

// Bed elevation at the nodes of one level block (node q = b n + a of a cell
// at (x0 + (i + x_a) dx, y0 + (j + x_b) dx)), bilinear in the raster
// g[jr][ir] at (gx0 + ir gdx, gy0 + jr gdy), clamped to its edge.
__global__ void k_amr_raster(RasterArgs A) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int n = A.n;
  if (t >= (size_t)A.ncell * n * n) return;
  const int cl = (int)(t / ((size_t)n * n)), q = (int)(t % ((size_t)n * n));
  const int a = q % n, b = q / n, cell = A.cell0 + cl;
  const double dx = A.cdx[cell];
  const int m = A.cmem[cell];
  const double x = A.mxy[m] + (A.ci[cell] + A.xh[a]) * dx;
  const double y = A.mxy[A.M + m] + (A.cj[cell] + A.xh[b]) * dx;
  const double fx = fmin(fmax((x - A.gx0) / A.gdx, 0.0), (double)(A.gnx - 1));
  const double fy = fmin(fmax((y - A.gy0) / A.gdy, 0.0), (double)(A.gny - 1));
  const int i0 = min((int)floor(fx), A.gnx - 2), j0 = min((int)floor(fy), A.gny - 2);
  const double tx = fx - i0, ty = fy - j0;
  const double* g = A.g + (size_t)j0 * A.gnx + i0;
  A.braw[A.off + t] = (1.0 - tx) * (1.0 - ty) * g[0] + tx * (1.0 - ty) * g[1] + (1.0 - tx) * ty * g[A.gnx] +
                      tx * ty * g[A.gnx + 1];
}

// Per cell: int h (eq:positivity-7) and int z_b l (eq:mass-loss) on the sample
// rule, one wavefront per cell.
__global__ __launch_bounds__(kAmrLanes) void k_amr_mass(AmrMassArgs A) {
  const int cl = blockIdx.x;
  if (cl >= A.ncell) return;
  const int cell = A.cell0 + cl, N1 = A.N1, NP = N1 * N1, S = A.S;
  __shared__ double s[16];
  for (int k = threadIdx.x; k < NP; k += blockDim.x) s[k] = A.z[(size_t)cell * NP + k];
  __syncthreads();
  double m = 0.0, zl = 0.0;
  for (int q = threadIdx.x; q < S * S; q += blockDim.x) {
    const int a = q % S, b = q / S;
    double z = 0.0;
    for (int jy = 0; jy < N1; ++jy)
      for (int jx = 0; jx < N1; ++jx) z += A.l[a * N1 + jx] * A.l[b * N1 + jy] * s[jy * N1 + jx];
    const double zb = A.zb[((size_t)cl * S + a) * S + b];
    const double w = A.w[a] * A.w[b];
    const double sd = z + zb;
    if (sd > 0.0) {
      m += w * sd;
      zl += w * zb;
    }
  }
  m = wave_sum(m);
  zl = wave_sum(zl);
  if (threadIdx.x == 0) {
    const double dx = A.cdx[cell];
    A.out[2 * (size_t)cell] = m * dx * dx;
    A.out[2 * (size_t)cell + 1] = zl * dx * dx;
  }
}

// Sum of the per-cell pairs in a fixed order: one workgroup, strided partial
// sums, then a tree.
__global__ __launch_bounds__(1024) void k_amr_sum2(const double* v, int K, double* out) {
  __shared__ double s0[1024], s1[1024];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    a += v[2 * (size_t)k];
    b += v[2 * (size_t)k + 1];
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s0[threadIdx.x] += s0[threadIdx.x + h];
      s1[threadIdx.x] += s1[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s0[0];
    out[1] = s1[0];
  }
}

}  // namespace

hipError_t launch_amr_eta(const AmrEtaArgs& a, hipStream_t s) {
  if (a.ncell <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_amr_eta, dim3(a.ncell), dim3(kAmrLanes), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_amr_transfer(const AmrXferArgs& a, hipStream_t s) {
  const int64_t n = (int64_t)a.Kn * a.NP;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_amr_transfer, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_amr_raster(const RasterArgs& a, hipStream_t s) {
  const int64_t n = (int64_t)a.ncell * a.n * a.n;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_amr_raster, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_amr_mass(const AmrMassArgs& a, hipStream_t s) {
  if (a.ncell <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_amr_mass, dim3(a.ncell), dim3(kAmrLanes), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_amr_sum2(const double* v, int K, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_amr_sum2, dim3(1), dim3(1024), 0, s, v, K, out);
  return hipGetLastError();
}

}  // namespace swk
