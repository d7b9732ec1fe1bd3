// Element-kernel instantiations for degree r = 1.
#include "sw_stage.inc"

namespace swk {

template <int P>
static hipError_t stage_p(int mode, const StageArgs& a, int nblk, hipStream_t s) {
  switch (mode) {
    case M_APPLY: hipLaunchKernelGGL((k_stage<1, P, M_APPLY>), dim3(nblk), dim3(kWave), 0, s, a); break;
    case M_FOLD: hipLaunchKernelGGL((k_stage<1, P, M_FOLD>), dim3(nblk), dim3(kWave), 0, s, a); break;
    case M_START: hipLaunchKernelGGL((k_stage<1, P, M_START>), dim3(nblk), dim3(kWave), 0, s, a); break;
    case M_STAGE: hipLaunchKernelGGL((k_stage<1, P, M_STAGE>), dim3(nblk), dim3(kWave), 0, s, a); break;
    case M_FINAL: hipLaunchKernelGGL((k_stage<1, P, M_FINAL>), dim3(nblk), dim3(kWave), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int P, int WPB, int IMEX = 0>
static hipError_t elem_pw(int mode, const StageArgs& a, int nblk, hipStream_t s) {
  switch (mode) {
    case F_START: hipLaunchKernelGGL((k_elem<1, P, F_START, WPB, IMEX>), dim3(nblk), dim3(WPB * kWave), 0, s, a); break;
    case F_STAGE: hipLaunchKernelGGL((k_elem<1, P, F_STAGE, WPB, IMEX>), dim3(nblk), dim3(WPB * kWave), 0, s, a); break;
    case F_FINAL: hipLaunchKernelGGL((k_elem<1, P, F_FINAL, WPB, IMEX>), dim3(nblk), dim3(WPB * kWave), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// wavefronts per workgroup: 1, 2 or 4 (cells per workgroup = wpb * 64 / P)
template <int P>
static hipError_t elem_p(int mode, int wpb, const StageArgs& a, int nblk, hipStream_t s) {
  if (a.imex) return wpb == 1 ? elem_pw<P, 1, 1>(mode, a, nblk, s) : hipErrorInvalidValue;
  switch (wpb) {
    case 1: return elem_pw<P, 1>(mode, a, nblk, s);
    case 2: return elem_pw<P, 2>(mode, a, nblk, s);
    case 4: return elem_pw<P, 4>(mode, a, nblk, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_stage_r1(int P, int mode, const StageArgs& a, int nblk, hipStream_t s) {
  switch (P) {
    case 4: return stage_p<4>(mode, a, nblk, s);
    case 8: return stage_p<8>(mode, a, nblk, s);
    case 16: return stage_p<16>(mode, a, nblk, s);
    case 32: return stage_p<32>(mode, a, nblk, s);
  }
  return hipErrorInvalidValue;
}

template <int P>
static hipError_t stage_scan_p(int mode, int mode2, const StageArgs& a, int nblk, hipStream_t s) {
  if (mode == M_START && mode2 < 0)
    hipLaunchKernelGGL((k_stage_scan<1, P, M_START, -1>), dim3(nblk), dim3(kWave), 0, s, a);
  else if (mode == M_STAGE && mode2 < 0)
    hipLaunchKernelGGL((k_stage_scan<1, P, M_STAGE, -1>), dim3(nblk), dim3(kWave), 0, s, a);
  else if (mode == M_FINAL && mode2 == M_START)
    hipLaunchKernelGGL((k_stage_scan<1, P, M_FINAL, M_START>), dim3(nblk), dim3(kWave), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_stage_scan_r1(int P, int mode, int mode2, const StageArgs& a, int nblk, hipStream_t s) {
  switch (P) {
    case 4: return stage_scan_p<4>(mode, mode2, a, nblk, s);
    case 8: return stage_scan_p<8>(mode, mode2, a, nblk, s);
    case 16: return stage_scan_p<16>(mode, mode2, a, nblk, s);
    case 32: return stage_scan_p<32>(mode, mode2, a, nblk, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_elem_r1(int P, int mode, int wpb, const StageArgs& a, int nblk, hipStream_t s) {
  switch (P) {
    case 4: return elem_p<4>(mode, wpb, a, nblk, s);
    case 8: return elem_p<8>(mode, wpb, a, nblk, s);
    case 16: return elem_p<16>(mode, wpb, a, nblk, s);
    case 32: return elem_p<32>(mode, wpb, a, nblk, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace swk
