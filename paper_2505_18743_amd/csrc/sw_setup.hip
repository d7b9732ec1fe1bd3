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
__global__ void k_cellinit(LevelTabs t, int cell0, int ncell, size_t off, int N1, const double* zb,
                           const double* cdx, double* bvec, double* zmax) {
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
  const double dx = cdx[cell0 + cl];
  bvec[(size_t)(cell0 + cl) * NP + i] = s * dx * dx;
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

__global__ void k_fill(double* p, size_t n, double v) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

__global__ void k_fill8(int8_t* p, size_t n, int8_t v) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

__global__ void k_copy8(const int8_t* a, int8_t* b, size_t n) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) b[t] = a[t];
}

__global__ void k_copy(const double* a, double* b, size_t n) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) b[t] = a[t];
}

__global__ void k_fill_n(double* p, int n, double v) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

// Minimum over a block of 256 threads (every thread gets the result).
__device__ double block_min(double m, double* sm) {
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + s]);
    __syncthreads();
  }
  const double r = sm[0];
  __syncthreads();
  return r;
}

// Chunk minimum: chunk b covers in[ch[2b] .. ch[2b] + ch[2b+1]) (at most 1024 items).
__global__ void k_minred_seg(const double* in, const int* ch, double* out) {
  __shared__ double sm[256];
  const int b0 = ch[2 * blockIdx.x], n = ch[2 * blockIdx.x + 1];
  double m = 1e300;
  for (int i = threadIdx.x; i < n; i += 256) m = fmin(m, in[b0 + i]);
  m = block_min(m, sm);
  if (threadIdx.x == 0) out[blockIdx.x] = m;
}

// Member minimum over its chunks [m0[m], m0[m+1]), times the member's CFL number
// (or 1 when cfl is NULL); one block per member.
__global__ void k_dt_seg(const double* part, const int* m0, const double* cfl, double* dst) {
  __shared__ double sm[256];
  const int m = blockIdx.x;
  double v = 1e300;
  for (int i = m0[m] + threadIdx.x; i < m0[m + 1]; i += 256) v = fmin(v, part[i]);
  v = block_min(v, sm);
  if (threadIdx.x == 0) dst[m] = (cfl ? cfl[m] : 1.0) * v;
}

// *dst = min(in[0..n)); one block.
__global__ void k_min_all(const double* in, int n, double* dst) {
  __shared__ double sm[256];
  double v = 1e300;
  for (int i = threadIdx.x; i < n; i += 256) v = fmin(v, in[i]);
  v = block_min(v, sm);
  if (threadIdx.x == 0) *dst = v;
}

__device__ void diag_combine(double* a, const double* b) {
  a[D_MINT] = fmin(a[D_MINT], b[D_MINT]);
  a[D_VIOL] += b[D_VIOL];
  a[D_NEWT] = fmax(a[D_NEWT], b[D_NEWT]);
  a[D_FALLB] += b[D_FALLB];
  a[D_MASS] += b[D_MASS];
  a[D_NR0] += b[D_NR0];
  a[D_NONF] = fmax(a[D_NONF], b[D_NONF]);
}

// Tree reduction of per-thread diagnostics over a block of 256 (fixed order);
// the result is left in s[.][0].
__device__ void block_diag(const double* v, double (*s)[256]) {
  const int t = threadIdx.x;
  for (int q = 0; q < D_NSLOT; ++q) s[q][t] = v[q];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (t < st) {
      double a[D_NSLOT], b[D_NSLOT];
      for (int q = 0; q < D_NSLOT; ++q) {
        a[q] = s[q][t];
        b[q] = s[q][t + st];
      }
      diag_combine(a, b);
      for (int q = 0; q < D_NSLOT; ++q) s[q][t] = a[q];
    }
    __syncthreads();
  }
}

// Per-cell diagnostics of one cell chunk (at most 256 cells of one member) ->
// chunk partials.
__global__ void k_diag_part_seg(const double* cdiag, const int8_t* flag, const int* ch, double* part) {
  __shared__ double s[D_NSLOT][256];
  const int t = threadIdx.x;
  const int c0 = ch[2 * blockIdx.x], n = ch[2 * blockIdx.x + 1];
  double v[D_NSLOT] = {1e300, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (t < n) {
    const int c = c0 + t;
    const double* d = cdiag + (size_t)c * D_NSLOT;
    v[D_MINT] = d[D_MINT];
    v[D_VIOL] = d[D_VIOL];
    v[D_NEWT] = d[D_NEWT];
    v[D_FALLB] = d[D_FALLB];
    v[D_MASS] = d[D_MASS];
    v[D_NR0] = flag[c] == 0 ? 1.0 : 0.0;
    v[D_NONF] = d[D_NONF];
  }
  block_diag(v, s);
  if (t == 0)
    for (int q = 0; q < D_NSLOT; ++q) part[(size_t)blockIdx.x * D_NSLOT + q] = s[q][0];
}

// End of step, one block per member: reduce the member's chunk partials in a
// fixed order into mdiag[m][0..D_NSLOT), record dt and advance the member's time.
__global__ void k_diag_seg(const double* part, const int* m0, double* mdiag, double* mt, const double* mdt) {
  __shared__ double s[D_NSLOT][256];
  const int t = threadIdx.x, m = blockIdx.x;
  double v[D_NSLOT] = {1e300, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = m0[m] + t; i < m0[m + 1]; i += 256) diag_combine(v, part + (size_t)i * D_NSLOT);
  block_diag(v, s);
  if (t == 0) {
    double* d = mdiag + (size_t)m * 16;
    for (int q = 0; q < D_NSLOT; ++q) d[q] = s[q][0];
    d[7] = mdt[m];
    mt[m] += mdt[m];
    d[8] = mt[m];
  }
}

}  // namespace swk
