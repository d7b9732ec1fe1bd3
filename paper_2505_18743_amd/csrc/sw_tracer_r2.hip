// Fast tracer kernel instantiations for degree r = 2.
#include "sw_tracer.inc"

namespace swk {

hipError_t launch_trc_r2(int P, int mode, const StageArgs& a, int nblk, hipStream_t s) {
  return trc_r<2>(P, mode, a, nblk, s);
}

hipError_t launch_trc_multi_r2(int P, int mode, const StageArgs& a, const TrcSet& ts, int nblk, hipStream_t s) {
  return trc_multi_r<2>(P, mode, a, ts, nblk, s);
}

hipError_t launch_trc_degree_r2(int P, const StageArgs& a, int nblk, hipStream_t s) {
  return trc_degree_r<2>(P, a, nblk, s);
}

}  // namespace swk
