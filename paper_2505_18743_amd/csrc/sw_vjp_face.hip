// Face part of the vector-Jacobian product of the weak residuals (gfx950, FP64),
// and the small kernels of the step adjoint.
//
// Same mapping as the forward face kernel: kFaceLanes lanes per face splitting
// the face nodes; the forward numerical flux (hydrostatic reconstruction,
// eq:hydro_rec_vars; Rusanov speed, eq:lxf_parameter; pressure term,
// eq:discharge_rhs) is recomputed at each node and differentiated in reverse
// order.  The state adjoints of the face rows are summed over the face's lanes
// and added into the adjoint arrays; one launch holds one face class, whose
// faces touch disjoint (cell, dof) sets, so no atomics are needed.  The bed
// offset adjoint of each face side goes to a per-face slot and is gathered per
// cell in a fixed order afterwards.
#include "sw_dev.h"

namespace swk {

template <int R>
__device__ __forceinline__ int vrow_dof(int side, int k) {
  constexpr int N1 = R + 1;
  return side == 0 ? k * N1 : side == 1 ? k * N1 + R : side == 2 ? k : R * N1 + k;
}

__device__ __forceinline__ void inv_des_d(double h, double eps, double& ih, double& dih) {
  if (!(h > 0.0)) {
    ih = 0.0;
    dih = 0.0;   // only reached through a dry clamp, whose derivative is 0
  } else if (h >= eps) {
    ih = 1.0 / h;
    dih = -ih * ih;
  } else {
    const double h4 = (h * h) * (h * h), e4 = (eps * eps) * (eps * eps);
    const double rs = 1.0 / sqrt(e4 + h4);
    ih = 1.4142135623730951 * h * rs;
    dih = 1.4142135623730951 * (e4 - h4) * rs * rs * rs;
  }
}

// Reverse pass of the face flux at one node.  cA, cB: adjoints of the values
// added to the A-side and B-side residuals (face weight included).  Outputs
// the adjoints of both traces (zeta, qx, qy) and of both depth samples.
__device__ __forceinline__ void flux_vjp(const double* vA, const double* vB, double zA, double zB, double nx,
                                         double ny, double g, double eps, const double* cA, const double* cB,
                                         double* gA, double* gB, double& gzA, double& gzB) {
  const double sAw = vA[0] + zA, sBw = vB[0] + zB;
  const double hA = sAw > 0.0 ? sAw : 0.0, hB = sBw > 0.0 ? sBw : 0.0;
  double ihA, dihA, ihB, dihB;
  inv_des_d(hA, eps, ihA, dihA);
  inv_des_d(hB, eps, ihB, dihB);
  const double uxA = vA[1] * ihA, uyA = vA[2] * ihA, uxB = vB[1] * ihB, uyB = vB[2] * ihB;
  const double unA = uxA * nx + uyA * ny, unB = uxB * nx + uyB * ny;
  const double cAw = hA > 0.0 ? sqrt(g * hA) : 0.0, cBw = hB > 0.0 ? sqrt(g * hB) : 0.0;
  const double lA = fabs(unA) + cAw, lB = fabs(unB) + cBw;
  const bool selA = lA >= lB;
  const double lam = selA ? lA : lB;
  const bool zsA = zA <= zB;
  const double zs = zsA ? zA : zB;
  const double tsA = vA[0] + zs, tsB = vB[0] + zs;
  const double hsA = tsA > 0.0 ? tsA : 0.0, hsB = tsB > 0.0 ? tsB : 0.0;
  const double qsxA = hsA * uxA, qsyA = hsA * uyA, qsxB = hsB * uxB, qsyB = hsB * uyB;
  const bool eA = vA[0] >= -zs, eB = vB[0] >= -zs;
  const double esA = eA ? vA[0] : -zs, esB = eB ? vB[0] : -zs;

  // adjoints of mass, momx, momy and the pressure term
  const double mb = cB[0] - cA[0], mxb = cB[1] - cA[1], myb = cB[2] - cA[2];
  const double pb = (cA[1] + cB[1]) * nx + (cA[2] + cB[2]) * ny;
  double qsxAb = 0.5 * nx * mb, qsxBb = 0.5 * nx * mb, qsyAb = 0.5 * ny * mb, qsyBb = 0.5 * ny * mb;
  double lamb = 0.5 * (esA - esB) * mb;
  double esAb = 0.5 * lam * mb, esBb = -0.5 * lam * mb;
  qsxAb += 0.5 * (unA + lam) * mxb;
  qsxBb += 0.5 * (unB - lam) * mxb;
  double unAb = 0.5 * qsxA * mxb, unBb = 0.5 * qsxB * mxb;
  lamb += 0.5 * (qsxA - qsxB) * mxb;
  qsyAb += 0.5 * (unA + lam) * myb;
  qsyBb += 0.5 * (unB - lam) * myb;
  unAb += 0.5 * qsyA * myb;
  unBb += 0.5 * qsyB * myb;
  lamb += 0.5 * (qsyA - qsyB) * myb;
  const double pg = 0.25 * g * pb;
  double hsAb = pg * (esA - esB), hsBb = pg * (esA - esB);
  esAb += pg * (hsA + hsB);
  esBb -= pg * (hsA + hsB);
  // q* = h* u
  hsAb += uxA * qsxAb + uyA * qsyAb;
  hsBb += uxB * qsxBb + uyB * qsyBb;
  double uxAb = hsA * qsxAb, uyAb = hsA * qsyAb, uxBb = hsB * qsxBb, uyBb = hsB * qsyBb;
  // zeta* = max(zeta, -z*), h* = max(zeta + z*, 0), z* = min(zA, zB)
  double zAb = 0.0, zBb = 0.0, zsb = 0.0;
  if (eA) zAb += esAb;
  else zsb -= esAb;
  if (eB) zBb += esBb;
  else zsb -= esBb;
  if (tsA > 0.0) {
    zAb += hsAb;
    zsb += hsAb;
  }
  if (tsB > 0.0) {
    zBb += hsBb;
    zsb += hsBb;
  }
  gzA = zsA ? zsb : 0.0;
  gzB = zsA ? 0.0 : zsb;
  // lam = max(|unA| + sqrt(g hA), |unB| + sqrt(g hB))
  const double lAb = selA ? lamb : 0.0, lBb = selA ? 0.0 : lamb;
  unAb += (unA > 0.0 ? 1.0 : (unA < 0.0 ? -1.0 : 0.0)) * lAb;
  unBb += (unB > 0.0 ? 1.0 : (unB < 0.0 ? -1.0 : 0.0)) * lBb;
  double hAb = cAw > 0.0 ? lAb * 0.5 * g / cAw : 0.0;
  double hBb = cBw > 0.0 ? lBb * 0.5 * g / cBw : 0.0;
  uxAb += nx * unAb;
  uyAb += ny * unAb;
  uxBb += nx * unBb;
  uyBb += ny * unBb;
  // u = q / h_des
  gA[1] = ihA * uxAb;
  gA[2] = ihA * uyAb;
  gB[1] = ihB * uxBb;
  gB[2] = ihB * uyBb;
  hAb += dihA * (vA[1] * uxAb + vA[2] * uyAb);
  hBb += dihB * (vB[1] * uxBb + vB[2] * uyBb);
  // h = max(zeta + zb, 0)
  if (sAw > 0.0) {
    zAb += hAb;
    gzA += hAb;
  }
  if (sBw > 0.0) {
    zBb += hBb;
    gzB += hBb;
  }
  gA[0] = zAb;
  gB[0] = zBb;
}

template <int R, int Q>
__global__ __launch_bounds__(kWave) void k_vjp_face(VjpFaceArgs A) {
  constexpr int N1 = R + 1, NP = N1 * N1, FPB = kWave / Q;
  const int S = A.S;
  const int tid = threadIdx.x, lane = tid % Q, lf = tid / Q;
  const int fl = blockIdx.x * FPB + lf;
  const bool fv = fl < A.nface;
  const int flc = fv ? fl : 0;
  const int f = A.face0 + flc;
  int cA = A.fA[f], cB = A.fB[f];
  const int meta = A.meta[f];
  const int sA = meta & 3, sB = (meta >> 2) & 3, sub = ((meta >> 4) & 3) - 1;
  const int bnd = (meta >> 6) & 1, bc = (meta >> 8) & 7;
  const bool ok = (cA >= 0 && cA < A.K) && (bnd || (cB >= 0 && cB < A.K));
  if (!ok && fv && lane == 0) atomicOr(A.err, 2);
  const bool act = fv && ok;
  if (!ok) cA = cB = 0;
  if (bnd) cB = cA;

  double cfA[3][N1], cfB[3][N1], rbA[3][N1], rbB[3][N1];
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      cfA[q][k] = A.u[q][(size_t)cA * NP + vrow_dof<R>(sA, k)];
      cfB[q][k] = A.u[q][(size_t)cB * NP + vrow_dof<R>(sB, k)];
      rbA[q][k] = A.rb[q][(size_t)cA * NP + vrow_dof<R>(sA, k)];
      rbB[q][k] = bnd ? 0.0 : A.rb[q][(size_t)cB * NP + vrow_dof<R>(sB, k)];
    }
  const double nx = sA == 0 ? -1.0 : (sA == 1 ? 1.0 : 0.0);
  const double ny = sA == 2 ? -1.0 : (sA == 3 ? 1.0 : 0.0);
  const double g = A.g, eps = A.eps;
  const double dxA = A.cdx[cA];
  const double* tB0 = A.fl + (size_t)(sub < 0 ? 0 : 1 + sub) * S * N1;
  double zeta_b = 0.0;
  if (bnd && bc == 1) {
    const double* td = A.mtide + (size_t)A.cmem[cA] * 4;
    zeta_b = td[0] * sin(6.283185307179586 * A.tt / td[1] + td[2]);
  }
  const double* gd = nullptr;
  if (bnd && (bc == 4 || bc == 5)) {
    const int go = A.gof[f];
    if (go >= 0 && go + S <= A.ng) gd = A.ghost + go;
    else if (fv && lane == 0) atomicOr(A.err, 2);
  }

  double gAk[3][N1], gBk[3][N1];
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int k = 0; k < N1; ++k) gAk[q][k] = gBk[q][k] = 0.0;
  double dAs = 0.0, dBs = 0.0;
#pragma unroll 1
  for (int al = lane; al < S; al += Q) {
    double la[N1], lb[N1];
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      la[k] = A.fl[al * N1 + k];
      lb[k] = tB0[al * N1 + k];
    }
    double vA[3], vB[3], cbA[3], cbB[3];
    const double wl = A.w[al] * dxA;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      double sa = 0.0, sb = 0.0, ra = 0.0, rb = 0.0;
#pragma unroll
      for (int k = 0; k < N1; ++k) {
        sa += la[k] * cfA[q][k];
        sb += lb[k] * cfB[q][k];
        ra += la[k] * rbA[q][k];
        rb += lb[k] * rbB[q][k];
      }
      vA[q] = sa;
      vB[q] = sb;
      cbA[q] = wl * ra;
      cbB[q] = wl * rb;
    }
    const double zA = A.zf[((size_t)flc * 2 + 0) * S + al];
    double zB = A.zf[((size_t)flc * 2 + 1) * S + al];
    if (bnd) {
      zB = zA;
      if (bc == 0) {
        const double qn = vA[1] * nx + vA[2] * ny;
        vB[0] = vA[0];
        vB[1] = vA[1] - 2.0 * qn * nx;
        vB[2] = vA[2] - 2.0 * qn * ny;
      } else if (bc == 1) {
        vB[0] = zeta_b;
        vB[1] = vA[1];
        vB[2] = vA[2];
      } else if (bc == 4 && gd) {
#pragma unroll
        for (int q = 0; q < 3; ++q) vB[q] = gd[(size_t)q * A.ng + al];
      } else if (bc == 5 && gd) {
        vB[0] = vA[0];
        vB[1] = gd[(size_t)1 * A.ng + al];
        vB[2] = gd[(size_t)2 * A.ng + al];
      } else {
        vB[0] = vA[0];
        vB[1] = vA[1];
        vB[2] = vA[2];
      }
    }
    double gA[3], gB[3], gzA, gzB;
    flux_vjp(vA, vB, zA, zB, nx, ny, g, eps, cbA, cbB, gA, gB, gzA, gzB);
    if (bnd) {
      // ghost state as a function of the interior trace
      if (bc == 0) {
        const double qn = gB[1] * nx + gB[2] * ny;
        gA[0] += gB[0];
        gA[1] += gB[1] - 2.0 * qn * nx;
        gA[2] += gB[2] - 2.0 * qn * ny;
      } else if (bc == 1) {
        gA[1] += gB[1];
        gA[2] += gB[2];
      } else if (bc == 4) {
        // given state: no dependence on the interior
      } else if (bc == 5) {
        gA[0] += gB[0];
      } else {
        gA[0] += gB[0];
        gA[1] += gB[1];
        gA[2] += gB[2];
      }
      gzA += gzB;
      gzB = 0.0;
    }
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int k = 0; k < N1; ++k) {
        gAk[q][k] += la[k] * gA[q];
        gBk[q][k] += lb[k] * gB[q];
      }
    dAs += gzA;
    dBs += gzB;
  }
  const size_t KN = (size_t)A.K * NP;
  (void)KN;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      const double va = gsum<Q>(gAk[q][k]);
      const double vb = gsum<Q>(gBk[q][k]);
      const int ia = q * N1 + k;
      if (act && (ia % Q) == lane) A.ub[q][(size_t)cA * NP + vrow_dof<R>(sA, k)] += va;
      if (act && !bnd && ((ia + 1) % Q) == lane) A.ub[q][(size_t)cB * NP + vrow_dof<R>(sB, k)] += vb;
    }
  }
  dAs = gsum<Q>(dAs);
  dBs = gsum<Q>(dBs);
  if (fv && lane == 0) {
    // zb = -(b + db): d zb / d db = -1
    A.fdb[2 * (size_t)f] = act ? -dAs : 0.0;
    A.fdb[2 * (size_t)f + 1] = (act && !bnd) ? -dBs : 0.0;
  }
}

template <int R>
static hipError_t vjp_face_r(const VjpFaceArgs& a, int nblk, hipStream_t s) {
  hipLaunchKernelGGL((k_vjp_face<R, kFaceLanes>), dim3(nblk), dim3(kWave), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_vjp_face(int r, const VjpFaceArgs& a, int nblk, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  switch (r) {
    case 1: return vjp_face_r<1>(a, nblk, s);
    case 2: return vjp_face_r<2>(a, nblk, s);
    case 3: return vjp_face_r<3>(a, nblk, s);
  }
  return hipErrorInvalidValue;
}

// dbbar[c] += sum of the per-face parts listed for cell c (fixed order).
__global__ void k_gather_fdb(const double* fdb, const int* off, const int* ent, int K, double* dbbar) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= K) return;
  double s = 0.0;
  for (int e = off[c]; e < off[c + 1]; ++e) s += fdb[ent[e]];
  dbbar[c] += s;
}

// state adjoint of the step: sb[f] += sum_l res[slot l][f], l < ns.
__global__ void k_vjp_combine(double* sb0, double* sb1, double* sb2, const double* res, int ns, size_t KN) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= KN) return;
  double* sb[3] = {sb0, sb1, sb2};
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    double v = sb[f][i];
    for (int l = 0; l < ns; ++l) v += res[((size_t)l * 4 + f) * KN + i];
    sb[f][i] = v;
  }
}

}  // namespace swk
