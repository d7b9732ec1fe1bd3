// Volume VJP kernel instantiations for degree r = 3.
#include "sw_vjp.inc"

namespace swk {

template <int P>
static hipError_t vjp_p(int mode, const VjpArgs& a, int nblk, hipStream_t s) {
  switch (mode) {
    case V_OP: hipLaunchKernelGGL((k_vjp_vol<3, P, V_OP>), dim3(nblk), dim3(kWave), 0, s, a); break;
    case V_STEP: hipLaunchKernelGGL((k_vjp_vol<3, P, V_STEP>), dim3(nblk), dim3(kWave), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_vjp_vol_r3(int P, int mode, const VjpArgs& a, int nblk, hipStream_t s) {
  switch (P) {
    case 4: return vjp_p<4>(mode, a, nblk, s);
    case 8: return vjp_p<8>(mode, a, nblk, s);
    case 16: return vjp_p<16>(mode, a, nblk, s);
    case 32: return vjp_p<32>(mode, a, nblk, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace swk
