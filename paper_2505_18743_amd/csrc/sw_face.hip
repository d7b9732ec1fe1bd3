// Face kernel of the sub-grid DG shallow-water operator (gfx950, FP64).
//
// One face per group of Q lanes (2, 4 or 8); the lanes split the face nodes (the
// fine or equal side's closed S-point rule, whose nodes are the boundary row of
// that side's sample grid).  At each node both traces come from the (r+1)
// nodal coefficients of the face row (GLL support points include the element
// end points, so the trace depends on that row only); hydrostatic
// reconstruction (eq:hydro_rec, eq:hydro_rec_vars) and the Rusanov flux
// (eq:lxf_parameter) give the flux, and the projections onto the (r+1) face
// test functions of each side are summed in registers, finished over the
// face's lanes with DPP moves and added into the stage's residual slot.  The
// faces of one launch touch disjoint (cell, dof) sets (one face class per
// launch), so no floating-point atomics are needed.
#include "sw_dev.h"

namespace swk {

template <int R>
__device__ __forceinline__ int row_dof(int side, int k) {
  constexpr int N1 = R + 1;
  return side == 0 ? k * N1 : side == 1 ? k * N1 + R : side == 2 ? k : R * N1 + k;
}

// NQ: 3 (flow), 4 (flow and tracer), or 1: the tracer's terms only, from the
// traces of all four fields (a tracer replay, whose flow is given)
template <int R, int Q, int NQ>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(R <= 2 ? 3 : 2))) void k_face(FaceArgs A) {
  constexpr int N1 = R + 1, NP = N1 * N1, FPB = kWave / Q;
  constexpr bool TO = NQ == 1;
  constexpr int NL = TO ? 4 : NQ;   // fields whose traces are read
  const int tid = threadIdx.x, lane = tid % Q, lf = tid / Q;
  const int bl = A.xmap ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  // segment of this workgroup (uniform); a single-segment launch (one level)
  // reads its parameters at fixed offsets, without the dependent lookup
  int sg = 0;
  if (A.nseg > 1)
    while (sg + 1 < A.nseg && bl >= A.sblk[sg + 1]) ++sg;
  const bool one = A.nseg == 1;
  const int S = one ? A.sS[0] : A.sS[sg];
  const double* flt = one ? A.sfl[0] : A.sfl[sg];
  const double* wt = one ? A.sw[0] : A.sw[sg];
  const double* zf = one ? A.szf[0] : A.szf[sg];
  const int fl = (one ? bl : bl - A.sblk[sg]) * FPB + lf;
  const bool fv = fl < (one ? A.snface[0] : A.snface[sg]);
  const int flc = fv ? fl : 0;
  const int f = (one ? A.sface0[0] : A.sface0[sg]) + flc;
  int cA = A.fA[f], cB = A.fB[f];
  const int meta = A.meta[f];
  const int sA = meta & 3, sB = (meta >> 2) & 3, sub = ((meta >> 4) & 3) - 1;
  const int bnd = (meta >> 6) & 1, bc = (meta >> 8) & 7;
  const bool ok = (cA >= 0 && cA < A.K) && (bnd || (cB >= 0 && cB < A.K));
  if (!ok && fv && lane == 0) atomicOr(A.err, 2);
  const bool act = fv && ok;
  if (!ok) cA = cB = 0;
  if (bnd) cB = cA;
  // face-row coefficients of both sides (GLL support points include the end
  // points, so each trace is the 1-D interpolant of that row)
  double cfA[NL][N1], cfB[NL][N1];
#pragma unroll
  for (int q = 0; q < NL; ++q)
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      cfA[q][k] = A.st[q][(size_t)cA * NP + row_dof<R>(sA, k)];
      cfB[q][k] = A.st[q][(size_t)cB * NP + row_dof<R>(sB, k)];
    }
  const double nx = sA == 0 ? -1.0 : (sA == 1 ? 1.0 : 0.0);
  const double ny = sA == 2 ? -1.0 : (sA == 3 ? 1.0 : 0.0);
  const double g = A.g, eps = A.eps;
  const double dxA = A.cdx[cA];
  const double* tB0 = flt + (size_t)(sub < 0 ? 0 : 1 + sub) * S * N1;
  double zeta_b = 0.0, c_in = 0.0;
  // given boundary data (state: all of zeta, q, c; discharge: q and inflow c)
  const double* gd = nullptr;
  if (bnd && (bc == 4 || bc == 5)) {
    const int go = A.gof[f];
    if (go >= 0 && go + S <= A.ng) gd = A.ghost + go;
    else if (fv && lane == 0) atomicOr(A.err, 2);
  }
  if (bnd && bc == 1) {
    const int m = A.cmem[cA];
    const double* td = A.mtide + (size_t)m * 4;
    const double tt = A.cstage != 0.0 ? A.mt[m] + A.cstage * A.mdt[m] : A.mt[m];
    zeta_b = td[0] * sin(6.283185307179586 * tt / td[1] + td[2]);
    c_in = td[3];
  }

  double pA[NQ][N1], pB[NQ][N1];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int k = 0; k < N1; ++k) pA[q][k] = pB[q][k] = 0.0;
  double lmax = 0.0;
#pragma unroll 1
  for (int al = lane; al < S; al += Q) {
    double la[N1], lb[N1];
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      la[k] = flt[al * N1 + k];
      lb[k] = tB0[al * N1 + k];
    }
    double vA[4] = {0.0, 0.0, 0.0, 0.0}, vB[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      double sa = 0.0, sb = 0.0;
#pragma unroll
      for (int k = 0; k < N1; ++k) {
        sa += la[k] * cfA[q][k];
        sb += lb[k] * cfB[q][k];
      }
      vA[q] = sa;
      vB[q] = sb;
    }
    const double zA = zf[((size_t)flc * 2 + 0) * S + al];
    double zB = zf[((size_t)flc * 2 + 1) * S + al];
    if (bnd) {
      zB = zA;
      if (bc == 0) {            // wall: mirror the normal discharge
        const double qn = vA[1] * nx + vA[2] * ny;
        vB[0] = vA[0];
        vB[1] = vA[1] - 2.0 * qn * nx;
        vB[2] = vA[2] - 2.0 * qn * ny;
        vB[3] = vA[3];
      } else if (bc == 1) {     // imposed elevation (tide), q extrapolated
        vB[0] = zeta_b;
        vB[1] = vA[1];
        vB[2] = vA[2];
        vB[3] = (vA[1] * nx + vA[2] * ny) < 0.0 ? c_in : vA[3];
      } else if (bc == 4 && gd) {   // given state
#pragma unroll
        for (int q = 0; q < 4; ++q) vB[q] = gd[(size_t)q * A.ng + al];
      } else if (bc == 5 && gd) {   // given discharge, zeta extrapolated, c given on inflow
        vB[0] = vA[0];
        vB[1] = gd[(size_t)1 * A.ng + al];
        vB[2] = gd[(size_t)2 * A.ng + al];
        vB[3] = (vB[1] * nx + vB[2] * ny) < 0.0 ? gd[(size_t)3 * A.ng + al] : vA[3];
      } else {                  // open: copy
#pragma unroll
        for (int q = 0; q < 4; ++q) vB[q] = vA[q];
      }
    }
    const double sAw = vA[0] + zA, sBw = vB[0] + zB;
    const double hA = sAw > 0.0 ? sAw : 0.0, hB = sBw > 0.0 ? sBw : 0.0;
    const double ihA = hA >= eps ? rcp_nr(hA) : inv_des(hA, eps);
    const double ihB = hB >= eps ? rcp_nr(hB) : inv_des(hB, eps);
    const double uxA = vA[1] * ihA, uyA = vA[2] * ihA, uxB = vB[1] * ihB, uyB = vB[2] * ihB;
    const double unA = uxA * nx + uyA * ny, unB = uxB * nx + uyB * ny;
    const double ghA = g * hA, ghB = g * hB;
    const double lA = fabs(unA) + (ghA > 0.0 ? ghA * rsq_nr(ghA) : 0.0);
    const double lB = fabs(unB) + (ghB > 0.0 ? ghB * rsq_nr(ghB) : 0.0);
    const double lam = lA >= lB ? lA : lB;
    const double zs = zA <= zB ? zA : zB;                       // z*_b = min(zb-, zb+)
    const double tsA = vA[0] + zs, tsB = vB[0] + zs;
    const double hsA = tsA > 0.0 ? tsA : 0.0, hsB = tsB > 0.0 ? tsB : 0.0;
    const double qsxA = hsA * uxA, qsyA = hsA * uyA, qsxB = hsB * uxB, qsyB = hsB * uyB;
    const double esA = vA[0] >= -zs ? vA[0] : -zs, esB = vB[0] >= -zs ? vB[0] : -zs;
    const double mass = 0.5 * ((qsxA + qsxB) * nx + (qsyA + qsyB) * ny) + 0.5 * lam * (esA - esB);
    const double momx = 0.5 * (qsxA * unA + qsxB * unB) + 0.5 * lam * (qsxA - qsxB);
    const double momy = 0.5 * (qsyA * unA + qsyB * unB) + 0.5 * lam * (qsyA - qsyB);
    const double pres = 0.5 * g * 0.5 * (hsA + hsB) * (esA - esB);
    const double trac = 0.5 * ((qsxA * vA[3] + qsxB * vB[3]) * nx + (qsyA * vA[3] + qsyB * vB[3]) * ny) +
                        0.5 * lam * (hsA * vA[3] - hsB * vB[3]);
    const double wl = wt[al] * dxA;
    const double cAv[4] = {-mass, -momx + pres * nx, -momy + pres * ny, -trac};
    const double cBv[4] = {mass, momx + pres * nx, momy + pres * ny, trac};
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int k = 0; k < N1; ++k) {
        pA[q][k] += wl * cAv[TO ? 3 : q] * la[k];
        pB[q][k] += wl * cBv[TO ? 3 : q] * lb[k];
      }
    lmax = fmax(lmax, lam);
  }
  // finish the face integrals over the face's lanes with a reduce-scatter
  // (lane l ends up owning entries l*PER .. l*PER + PER - 1 of each side),
  // then read all owned residual entries, add, and write them back; faces of
  // one launch touch disjoint (cell, dof) sets
  constexpr int NE = NQ * N1, NEP = ((NE + Q - 1) / Q) * Q, PER = NEP / Q;
  const size_t KN = (size_t)A.K * NP;
  double* rA = A.res + (size_t)A.slot * 4 * KN + (size_t)cA * NP;
  double* rB = A.res + (size_t)A.slot * 4 * KN + (size_t)cB * NP;
  double xa[NEP], xb[NEP];
#pragma unroll
  for (int i = 0; i < NEP; ++i) {
    xa[i] = i < NE ? pA[i / N1][i % N1] : 0.0;
    xb[i] = i < NE ? pB[i / N1][i % N1] : 0.0;
  }
  reduce_scatter<Q, NEP>(xa, lane);
  reduce_scatter<Q, NEP>(xb, lane);
  double* pa[PER];
  double* pb[PER];
  double oa[PER], ob[PER];
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int ia = lane * PER + e;
    const int iq = ia < NE ? ia / N1 : 0, ik = ia < NE ? ia % N1 : 0;
    const int fq = TO ? 3 : iq;   // the residual field of entry ia
    pa[e] = rA + (size_t)fq * KN + row_dof<R>(sA, ik);
    pb[e] = rB + (size_t)fq * KN + row_dof<R>(sB, ik);
    oa[e] = *pa[e];      // in range for every lane (clamped entry); used only if owned
    ob[e] = *pb[e];
  }
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int ia = lane * PER + e;
    if (act && ia < NE) *pa[e] = oa[e] + xa[e];
    if (act && !bnd && ia < NE) *pb[e] = ob[e] + xb[e];
  }
  // positivity time-step bound (Prop. 3.2): w J_K / (lambda l_Gamma) on both sides
  lmax = gmin<Q>(-lmax);
  lmax = -lmax;
  double bnd_dt = 1e300;
  if (act && lmax > 0.0) {
    bnd_dt = A.cw1[cA] * A.cdx[cA] * A.cdx[cA] / (lmax * dxA);
    if (!bnd) bnd_dt = fmin(bnd_dt, A.cw1[cB] * A.cdx[cB] * A.cdx[cB] / (lmax * dxA));
  }
  if (fv && lane == 0) A.fdt[f] = bnd_dt;
}

template <int R, int Q>
static hipError_t face_rq(const FaceArgs& a, int nblk, hipStream_t s) {
  if (a.tracer && a.tonly) hipLaunchKernelGGL((k_face<R, Q, 1>), dim3(nblk), dim3(kWave), 0, s, a);
  else if (a.tracer) hipLaunchKernelGGL((k_face<R, Q, 4>), dim3(nblk), dim3(kWave), 0, s, a);
  else hipLaunchKernelGGL((k_face<R, Q, 3>), dim3(nblk), dim3(kWave), 0, s, a);
  return hipGetLastError();
}

template <int R>
static hipError_t face_r(int q, const FaceArgs& a, int nblk, hipStream_t s) {
  switch (q) {
    case 2: return face_rq<R, 2>(a, nblk, s);
    case 4: return face_rq<R, 4>(a, nblk, s);
    case 8: return face_rq<R, 8>(a, nblk, s);
  }
  return hipErrorInvalidValue;
}

// q lanes per face (2, 4 or 8): 64 / q faces per workgroup
hipError_t launch_face(int r, int q, const FaceArgs& a, int nblk, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  switch (r) {
    case 1: return face_r<1>(q, a, nblk, s);
    case 2: return face_r<2>(q, a, nblk, s);
    case 3: return face_r<3>(q, a, nblk, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace swk
