// Fast tracer kernel instantiations for degree r = 1.
#include "sw_tracer.inc"

namespace swk {

hipError_t launch_trc_r1(int P, int mode, const StageArgs& a, int nblk, hipStream_t s) {
  return trc_r<1>(P, mode, a, nblk, s);
}

hipError_t launch_trc_multi_r1(int P, int mode, const StageArgs& a, const TrcSet& ts, int nblk, hipStream_t s) {
  return trc_multi_r<1>(P, mode, a, ts, nblk, s);
}

hipError_t launch_trc_degree_r1(int P, const StageArgs& a, int nblk, hipStream_t s) {
  return trc_degree_r<1>(P, a, nblk, s);
}

}  // namespace swk
