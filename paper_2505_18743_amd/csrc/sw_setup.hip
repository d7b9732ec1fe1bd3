// Setup and small bookkeeping kernels: bathymetry layout, face samples,
// per-cell precomputations, Definition 3.1 initial state, reductions.
#include "sw_dev.h"

namespace swk {

// ABI layout [cell][b][a] of bed elevation -> internal depth [cell][a][b],
// zb = -(b + db_K) (Sec. 2: h = zeta + z_b).
__global__ void k_bathy(const double* braw, const double* db, double* zb, int cell0, int ncell, int S, size_t off) {
  const size_t n = (size_t)ncell * S * S;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int cl = (int)(t / ((size_t)S * S));
  const int rem = (int)(t % ((size_t)S * S));
  const int b = rem / S, a = rem % S;
  zb[off + ((size_t)cl * S + a) * S + b] = -(braw[off + t] + db[cell0 + cl]);
}

__device__ __forceinline__ void row_node(int side, int al, int S, int& a, int& b) {
  if (side == 0) { a = 0; b = al; }
  else if (side == 1) { a = S - 1; b = al; }
  else if (side == 2) { a = al; b = 0; }
  else { a = al; b = S - 1; }
}

// Face samples of a level group: side A = its own boundary row; side B = its
// own row (conforming), the fine side's raw sample at the same point with the
// coarse cell's offset (hanging), or side A (boundary).
__global__ void k_facez(const int* fA, const int* fB, const int* meta, int face0, int nface, int S, int cell0,
                        int ncell, size_t off, const double* zb, const double* braw, const double* db, double* zf,
                        int* err, int K) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nface * S) return;
  const int fl = t / S, al = t % S;
  const int f = face0 + fl;
  const int cA = fA[f], cB = fB[f], m = meta[f];
  const int sA = m & 3, sB = (m >> 2) & 3, sub = ((m >> 4) & 3) - 1, bnd = (m >> 6) & 1;
  const bool cBok = bnd || (sub < 0 ? (cB >= cell0 && cB < cell0 + ncell) : (cB >= 0 && cB < K));
  if (cA < cell0 || cA >= cell0 + ncell || !cBok) {
    atomicOr(err, 4);
    return;
  }
  int a, b;
  row_node(sA, al, S, a, b);
  const size_t ia = off + ((size_t)(cA - cell0) * S + a) * S + b;
  const double za = zb[ia];
  double zbv;
  if (bnd) {
    zbv = za;
  } else if (sub < 0) {
    int a2, b2;
    row_node(sB, al, S, a2, b2);
    zbv = zb[off + ((size_t)(cB - cell0) * S + a2) * S + b2];
  } else {
    zbv = -(braw[off + (size_t)(cA - cell0) * S * S + (size_t)b * S + a] + db[cB]);
  }
  zf[((size_t)fl * 2 + 0) * S + al] = za;
  zf[((size_t)fl * 2 + 1) * S + al] = zbv;
}

// Per cell: max depth sample and the all-wet B_i = sum_q W_q psi_i(x_q) zb_q.
__global__ void k_cellinit(LevelTabs t, int cell0, int ncell, size_t off, int N1, const double* zb, double* bvec,
                           double* zmax) {
  const int NP = N1 * N1;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ncell * NP) return;
  const int cl = q / NP, i = q % NP;
  const int ix = i % N1, iy = i / N1;
  const int S = t.S;
  const double* z = zb + off + (size_t)cl * S * S;
  double s = 0.0, mx = -1e300;
  for (int a = 0; a < S; ++a) {
    double sa = 0.0;
    for (int b = 0; b < S; ++b) {
      const double zv = z[(size_t)a * S + b];
      sa += t.w[b] * t.l[b * N1 + iy] * zv;
      mx = fmax(mx, zv);
    }
    s += t.w[a] * t.l[a * N1 + ix] * sa;
  }
  bvec[(size_t)(cell0 + cl) * NP + i] = s * t.dx * t.dx;
  if (i == 0) zmax[cell0 + cl] = mx;
}

// Definition 3.1: keep eta where some sample node is wet, else -max zb; q = 0.
__global__ void k_lake(LevelTabs t, int cell0, int ncell, size_t off, int N1, const double* zb, const double* zmax,
                       const double* eta, double* zeta, double* qx, double* qy) {
  const int NP = N1 * N1;
  const int cl = blockIdx.x * blockDim.x + threadIdx.x;
  if (cl >= ncell) return;
  const int cell = cell0 + cl;
  const int S = t.S;
  const double* z = zb + off + (size_t)cl * S * S;
  bool wet = false;
  for (int a = 0; a < S && !wet; ++a)
    for (int b = 0; b < S; ++b) {
      double v = 0.0;
      for (int jy = 0; jy < N1; ++jy) {
        double r = 0.0;
        for (int jx = 0; jx < N1; ++jx) r += t.l[a * N1 + jx] * eta[(size_t)cell * NP + jy * N1 + jx];
        v += t.l[b * N1 + jy] * r;
      }
      if (v + z[(size_t)a * S + b] > 0.0) {
        wet = true;
        break;
      }
    }
  for (int j = 0; j < NP; ++j) {
    zeta[(size_t)cell * NP + j] = wet ? eta[(size_t)cell * NP + j] : -zmax[cell];
    qx[(size_t)cell * NP + j] = 0.0;
    qy[(size_t)cell * NP + j] = 0.0;
  }
}

__global__ void k_set(double* p, int i, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[i] = v;
}

__global__ void k_fill(double* p, size_t n, double v) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

__global__ void k_fill8(int8_t* p, size_t n, int8_t v) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

__global__ void k_copy(const double* a, double* b, size_t n) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) b[t] = a[t];
}

// Block-wise minimum: out[b] = min(in[b*1024 .. b*1024+1023]).
__global__ void k_minred(const double* in, int n, double* out) {
  __shared__ double sm[256];
  const int base = blockIdx.x * 1024 + threadIdx.x;
  double m = 1e300;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = base + u * 256;
    if (i < n) m = fmin(m, in[i]);
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sm[0];
}

// dt = cfl * min(in[0..n)) (or the fixed dt when fixed > 0); one block of 256.
__global__ void k_dt(const double* in, int n, double cfl, double fixed, double* dst) {
  __shared__ double sm[256];
  double m = 1e300;
  for (int i = threadIdx.x; i < n; i += 256) m = fmin(m, in[i]);
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *dst = fixed > 0.0 ? fixed : cfl * sm[0];
}

// Per-cell diagnostics -> per-block partials (256 cells per block).
__global__ void k_diag_part(const double* cdiag, const int8_t* flag, int K, double* part) {
  __shared__ double s[D_NSLOT][256];
  const int t = threadIdx.x;
  const int c = blockIdx.x * 256 + t;
  double v[D_NSLOT] = {1e300, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (c < K) {
    const double* d = cdiag + (size_t)c * D_NSLOT;
    v[D_MINT] = d[D_MINT];
    v[D_VIOL] = d[D_VIOL];
    v[D_NEWT] = d[D_NEWT];
    v[D_FALLB] = d[D_FALLB];
    v[D_MASS] = d[D_MASS];
    v[D_NR0] = flag[c] == 0 ? 1.0 : 0.0;
    v[D_NONF] = d[D_NONF];
  }
  for (int q = 0; q < D_NSLOT; ++q) s[q][t] = v[q];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (t < st) {
      s[D_MINT][t] = fmin(s[D_MINT][t], s[D_MINT][t + st]);
      s[D_VIOL][t] += s[D_VIOL][t + st];
      s[D_NEWT][t] = fmax(s[D_NEWT][t], s[D_NEWT][t + st]);
      s[D_FALLB][t] += s[D_FALLB][t + st];
      s[D_MASS][t] += s[D_MASS][t + st];
      s[D_NR0][t] += s[D_NR0][t + st];
      s[D_NONF][t] = fmax(s[D_NONF][t], s[D_NONF][t + st]);
    }
    __syncthreads();
  }
  if (t == 0)
    for (int q = 0; q < D_NSLOT; ++q) part[(size_t)blockIdx.x * D_NSLOT + q] = s[q][0];
}

// End of step: reduce the block partials in a fixed order and advance t.
__global__ void k_diag(const double* part, int n, double* diag, double* scal) {
  __shared__ double s[D_NSLOT][256];
  const int t = threadIdx.x;
  double v[D_NSLOT] = {1e300, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = t; i < n; i += 256) {
    const double* d = part + (size_t)i * D_NSLOT;
    v[D_MINT] = fmin(v[D_MINT], d[D_MINT]);
    v[D_VIOL] += d[D_VIOL];
    v[D_NEWT] = fmax(v[D_NEWT], d[D_NEWT]);
    v[D_FALLB] += d[D_FALLB];
    v[D_MASS] += d[D_MASS];
    v[D_NR0] += d[D_NR0];
    v[D_NONF] = fmax(v[D_NONF], d[D_NONF]);
  }
  for (int q = 0; q < D_NSLOT; ++q) s[q][t] = v[q];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (t < st) {
      s[D_MINT][t] = fmin(s[D_MINT][t], s[D_MINT][t + st]);
      s[D_VIOL][t] += s[D_VIOL][t + st];
      s[D_NEWT][t] = fmax(s[D_NEWT][t], s[D_NEWT][t + st]);
      s[D_FALLB][t] += s[D_FALLB][t + st];
      s[D_MASS][t] += s[D_MASS][t + st];
      s[D_NR0][t] += s[D_NR0][t + st];
      s[D_NONF][t] = fmax(s[D_NONF][t], s[D_NONF][t + st]);
    }
    __syncthreads();
  }
  if (t == 0) {
    for (int q = 0; q < D_NSLOT; ++q) diag[q] = s[q][0];
    diag[7] = scal[0];
    scal[1] += scal[0];
    diag[8] = scal[1];
  }
}

}  // namespace swk
