// Device helpers shared by the element and face kernels.
#pragma once
#include "sw_internal.h"

namespace swk {

// Cross-lane moves within groups of P consecutive lanes (P a power of two):
// DPP quad permutations and row mirrors (within 16 lanes), a ds_bpermute for
// the larger strides.  Every lane of a group takes part in the same call.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = dpp_i<CTRL>(__double2loint(v));
  const int hi = dpp_i<CTRL>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
// partner value for butterfly step m (m = 1, 2, 4, 8, 16, 32)
template <int M>
__device__ __forceinline__ double partner(double v) {
  if constexpr (M == 1) return dpp_d<0xB1>(v);        // quad_perm(1,0,3,2)
  else if constexpr (M == 2) return dpp_d<0x4E>(v);   // quad_perm(2,3,0,1)
  else if constexpr (M == 4) return dpp_d<0x141>(v);  // row_half_mirror
  else if constexpr (M == 8) return dpp_d<0x140>(v);  // row_mirror
  else return __shfl_xor(v, M);
}
template <int M>
__device__ __forceinline__ int partner_i(int v) {
  if constexpr (M == 1) return dpp_i<0xB1>(v);
  else if constexpr (M == 2) return dpp_i<0x4E>(v);
  else if constexpr (M == 4) return dpp_i<0x141>(v);
  else if constexpr (M == 8) return dpp_i<0x140>(v);
  else return __shfl_xor(v, M);
}
// Lane k's value (k a constant once the caller's loop is unrolled) to every
// lane of its group of P: the DPP broadcast of a row lane (P = 16; P = 8 takes
// two and keeps its half-row's) or of a quad lane (P = 4), a ds_bpermute
// otherwise.
template <int K>
__device__ __forceinline__ double row_bcast(double v) {
  return dpp_d<0x150 + K>(v);   // row_newbcast:K
}
template <int K>
__device__ __forceinline__ double quad_bcast(double v) {
  return dpp_d<K | (K << 2) | (K << 4) | (K << 6)>(v);   // quad_perm(K,K,K,K)
}
template <int P>
__device__ __forceinline__ double gbcast(double v, int k) {
  if constexpr (P == 16) {
    switch (k) {
      case 0: return row_bcast<0>(v);
      case 1: return row_bcast<1>(v);
      case 2: return row_bcast<2>(v);
      case 3: return row_bcast<3>(v);
      case 4: return row_bcast<4>(v);
      case 5: return row_bcast<5>(v);
      case 6: return row_bcast<6>(v);
      case 7: return row_bcast<7>(v);
      case 8: return row_bcast<8>(v);
      case 9: return row_bcast<9>(v);
      case 10: return row_bcast<10>(v);
      case 11: return row_bcast<11>(v);
      case 12: return row_bcast<12>(v);
      case 13: return row_bcast<13>(v);
      case 14: return row_bcast<14>(v);
      default: return row_bcast<15>(v);
    }
  } else if constexpr (P == 8) {
    // a row broadcast reaches 16 lanes: lane k for the lower half-row, lane
    // 8 + k for the upper
    double lo, hi;
    switch (k) {
      case 0: lo = row_bcast<0>(v); hi = row_bcast<8>(v); break;
      case 1: lo = row_bcast<1>(v); hi = row_bcast<9>(v); break;
      case 2: lo = row_bcast<2>(v); hi = row_bcast<10>(v); break;
      case 3: lo = row_bcast<3>(v); hi = row_bcast<11>(v); break;
      case 4: lo = row_bcast<4>(v); hi = row_bcast<12>(v); break;
      case 5: lo = row_bcast<5>(v); hi = row_bcast<13>(v); break;
      case 6: lo = row_bcast<6>(v); hi = row_bcast<14>(v); break;
      default: lo = row_bcast<7>(v); hi = row_bcast<15>(v); break;
    }
    return (__lane_id() & 8) ? hi : lo;
  } else if constexpr (P == 4) {
    switch (k) {
      case 0: return quad_bcast<0>(v);
      case 1: return quad_bcast<1>(v);
      case 2: return quad_bcast<2>(v);
      default: return quad_bcast<3>(v);
    }
  } else {
    return __shfl(v, k, P);
  }
}

// Ordering point for LDS data exchanged inside one wavefront (the wave's LDS
// operations complete in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exact xor partners inside a row of 16 lanes: the row mirror pairs i with
// 15 - i = i ^ 15, the half-row mirror i with i ^ 7 (within each 8 lanes).
template <int XM>
__device__ __forceinline__ double xpartner(double v) {
  if constexpr (XM == 1) return dpp_d<0xB1>(v);
  else if constexpr (XM == 2) return dpp_d<0x4E>(v);
  else if constexpr (XM == 7) return dpp_d<0x141>(v);
  else if constexpr (XM == 15) return dpp_d<0x140>(v);
  else return __shfl_xor(v, XM);
}

// One halving step of a reduce-scatter: a lane whose decision bit is set keeps
// the upper half of x[0..2H) and sends the lower half to its partner (which
// keeps the lower half); the kept half, summed with what the partner sent,
// moves to x[0..H).
template <int XM, int H>
__device__ __forceinline__ void rs_step(double* x, bool up) {
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const double send = up ? x[i] : x[H + i];
    const double keep = up ? x[H + i] : x[i];
    x[i] = keep + xpartner<XM>(send);
  }
}

// Sum of x[0..V) over the P lanes of a group (V a multiple of P), scattered:
// afterwards lane l (index within the group) holds the totals of entries
// l*(V/P) .. l*(V/P) + V/P - 1 in x[0..V/P).  The partners lane ^ 16, ^ 15,
// ^ 7, ^ 2, ^ 1 are taken from the high decision bit down, so partners always
// hold the same subset of entries and the pairings span all P lanes.
// Workgroup index remapped so that each of the 8 XCDs (workgroups are handed
// out round robin over them) takes one contiguous range of the grid, where
// neighbouring cells or faces share cache lines of the nodal blocks and the
// sample rows stream from nearby HBM pages.  A bijection of [0, n).
__device__ __forceinline__ int xcd_block(int b, int n) {
  constexpr int X = 8;
  const int q = n / X, rm = n % X, x = b % X, i = b / X;
  return x * q + (x < rm ? x : rm) + i;
}

template <int P, int V>
__device__ __forceinline__ void reduce_scatter(double* x, int lane) {
  static_assert(V % P == 0, "V must be a multiple of P");
  // at decision bit b the kept half has V * 2^b / P entries
  if constexpr (P >= 32) rs_step<16, V * 16 / P>(x, (lane >> 4) & 1);
  if constexpr (P >= 16) rs_step<15, V * 8 / P>(x, (lane >> 3) & 1);
  if constexpr (P >= 8) rs_step<7, V * 4 / P>(x, (lane >> 2) & 1);
  if constexpr (P >= 4) rs_step<2, V * 2 / P>(x, (lane >> 1) & 1);
  if constexpr (P >= 2) rs_step<1, V / P>(x, lane & 1);
}

// After the quad steps every lane of a quad holds the quad result, so the
// mirrors combine whole quads (half rows) exactly like an xor butterfly.
template <int P>
__device__ __forceinline__ double gsum(double v) {
  if constexpr (P >= 2) v += partner<1>(v);
  if constexpr (P >= 4) v += partner<2>(v);
  if constexpr (P >= 8) v += partner<4>(v);
  if constexpr (P >= 16) v += partner<8>(v);
  if constexpr (P >= 32) v += partner<16>(v);
  if constexpr (P >= 64) v += partner<32>(v);
  return v;
}
template <int P>
__device__ __forceinline__ double gmin(double v) {
  if constexpr (P >= 2) v = fmin(v, partner<1>(v));
  if constexpr (P >= 4) v = fmin(v, partner<2>(v));
  if constexpr (P >= 8) v = fmin(v, partner<4>(v));
  if constexpr (P >= 16) v = fmin(v, partner<8>(v));
  if constexpr (P >= 32) v = fmin(v, partner<16>(v));
  if constexpr (P >= 64) v = fmin(v, partner<32>(v));
  return v;
}
template <int P>
__device__ __forceinline__ int gand(int v) {
  if constexpr (P >= 2) v &= partner_i<1>(v);
  if constexpr (P >= 4) v &= partner_i<2>(v);
  if constexpr (P >= 8) v &= partner_i<4>(v);
  if constexpr (P >= 16) v &= partner_i<8>(v);
  if constexpr (P >= 32) v &= partner_i<16>(v);
  if constexpr (P >= 64) v &= partner_i<32>(v);
  return v;
}
template <int P>
__device__ __forceinline__ int gor(int v) {
  if constexpr (P >= 2) v |= partner_i<1>(v);
  if constexpr (P >= 4) v |= partner_i<2>(v);
  if constexpr (P >= 8) v |= partner_i<4>(v);
  if constexpr (P >= 16) v |= partner_i<8>(v);
  if constexpr (P >= 32) v |= partner_i<16>(v);
  if constexpr (P >= 64) v |= partner_i<32>(v);
  return v;
}

// 1/h_des of the desingularised velocity (eq:velocity)
__device__ __forceinline__ double inv_des(double h, double eps) {
  const double h4 = (h * h) * (h * h);
  const double e4 = (eps * eps) * (eps * eps);
  return 1.4142135623730951 * h / sqrt(fmax(h4, e4) + h4);
}

// The three iterations below start from an estimate with relative error
// |e| of order 1e-7 and apply one third-order correction, the series of
// (1 - e)^(-k) cut after e^2: the remaining error is of order e^3, below the
// rounding of a double, with fewer dependent steps than two Newton steps.

// 1/x for finite x > 0: hardware estimate y, e = 1 - x y, 1/x = y (1 + e + e^2 + ...).
__device__ __forceinline__ double rcp_nr(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, y, 1.0);
  return fma(y, fma(e, e, e), y);
}

// x^{-1/2} for finite x > 0: hardware estimate y, e = 1 - x y^2,
// x^{-1/2} = y (1 + e/2 + 3 e^2/8 + ...).
__device__ __forceinline__ double rsq_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}

// x^{-1/3} for finite x > 0: single-precision 2^{-log2(x)/3} as the start z,
// e = 1 - x z^3, x^{-1/3} = z (1 + e/3 + 2 e^2/9 + ...).
__device__ __forceinline__ double rcbrt_nr(double x) {
  const float xf = (float)x;
  const double z = (double)__builtin_amdgcn_exp2f(-__builtin_amdgcn_logf(xf) * 0.333333343f);
  const double e = fma(-x, z * z * z, 1.0);
  return fma(z * e, fma(e, 0.2222222222222222, 0.3333333333333333), z);
}

// Pointwise factors of the volume terms at one node: ih = 1/h_des (eq:velocity)
// and gam = g n^2 |q| h_des^{-7/3} (eq:manning with the desingularised depth).
// For h >= eps the definition gives h_des = h exactly, evaluated through the
// reciprocal and inverse-cube-root iterations; below eps (thin layers, dry
// nodes) the definition is evaluated as written.
__device__ __forceinline__ void pointwise(double h, double qx, double qy, double eps, double gn2, bool fric,
                                          double& ih, double& gam) {
  gam = 0.0;
  double hd;                     // h_des = 1/ih, the depth the friction law sees
  if (h >= eps) {
    ih = rcp_nr(h);
    hd = h;
  } else if (h > 0.0) {
    // below eps: ih = sqrt(2) h / sqrt(eps^4 + h^4) (the max picks eps^4)
    const double h2 = h * h, e2 = eps * eps;
    ih = 1.4142135623730951 * h * rsq_nr(fma(e2, e2, h2 * h2));
    hd = rcp_nr(ih);
  } else {
    ih = 0.0;                    // dry node: no velocity, no friction
    return;
  }
  if (fric) {
    const double q2 = qx * qx + qy * qy;
    const double qn = q2 > 0.0 ? q2 * rsq_nr(q2) : 0.0;
    gam = gn2 * qn * (ih * ih) * rcbrt_nr(hd);
  }
}

// gamma(|q|, h) = g n^2 |q| h^{-7/3} of eq:manning at the plain depth h, the
// coefficient of the friction-modified discharge matrix
// (eq:mass_matrix_discharge).  For h >= eps it equals the desingularised value
// gam_des that pointwise() returns (h_des = h there); below eps it is
// (1/h)^2 h^{-1/3}, with h scaled by an exact power of two before the cube
// root when it is below the range of the single-precision start; a dry node
// (h = 0) or a node without discharge gives zero.
__device__ __forceinline__ double gamma_plain(double h, double qx, double qy, double eps, double gn2, bool fric,
                                              double gam_des) {
  if (h >= eps) return gam_des;
  const double q2 = qx * qx + qy * qy;
  if (!fric || !(h > 0.0) || !(q2 > 0.0)) return 0.0;
  const double qn = q2 * rsq_nr(q2);
  const double ih = rcp_nr(h);
  const bool tiny = h < 0x1p-96;
  const double c = tiny ? rcbrt_nr(h * 0x1p96) * 0x1p32 : rcbrt_nr(h);
  return gn2 * qn * (ih * ih) * c;
}

// Round-off water of a dry cell: 64 u |z_max| |K| (u = 2^-52), the mass the
// scalar solve of Hbar = 0 can leave where zeta + z_b cancels to a few ulps
// of the largest depth sample.  A cell with no more water than this counts
// as dry for the tracer (its concentration is kept).
__device__ __forceinline__ double dry_floor(double zmax, double area) {
  return 0x1p-46 * fabs(zmax) * area;
}

}  // namespace swk
