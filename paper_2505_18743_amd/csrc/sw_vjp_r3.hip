// Volume VJP kernel instantiations for degree r = 3.
#include "sw_vjp.inc"

namespace swk {

hipError_t launch_vjp_vol_r3(int P, int mode, const VjpArgs& a, int nblk, hipStream_t s) {
  return vjp_r<3>(P, mode, a, nblk, s);
}

}  // namespace swk
