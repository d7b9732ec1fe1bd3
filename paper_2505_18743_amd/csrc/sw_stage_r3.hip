// Element-kernel instantiations for degree r = 3.
#include "sw_stage_dispatch.inc"

namespace swk {

hipError_t launch_stage_r3(int P, int mode, const StageArgs& a, int nblk, hipStream_t s) {
  return stage_r<3>(P, mode, a, nblk, s);
}

hipError_t launch_stage_scan_r3(int P, int mode, int mode2, const StageArgs& a, int nblk, hipStream_t s) {
  return stage_scan_r<3>(P, mode, mode2, a, nblk, s);
}

hipError_t launch_elem_r3(int P, int mode, int wpb, const StageArgs& a, int nblk, hipStream_t s) {
  return elem_r<3>(P, mode, wpb, a, nblk, s);
}

}  // namespace swk
