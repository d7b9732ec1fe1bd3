// Fast tracer kernel instantiations for degree r = 3.
#include "sw_tracer.inc"

namespace swk {

hipError_t launch_trc_r3(int P, int mode, const StageArgs& a, int nblk, hipStream_t s) {
  return trc_r<3>(P, mode, a, nblk, s);
}

hipError_t launch_trc_multi_r3(int P, int mode, const StageArgs& a, const TrcSet& ts, int nblk, hipStream_t s) {
  return trc_multi_r<3>(P, mode, a, ts, nblk, s);
}

hipError_t launch_trc_degree_r3(int P, const StageArgs& a, int nblk, hipStream_t s) {
  return trc_degree_r<3>(P, a, nblk, s);
}

}  // namespace swk
