// hh_batched.hip -- length-bucketed planner + persistent kernel (in progress:
// routes to the quad kernel until the planner lands).

#include "hh_device.hpp"
#include "hh_internal.hpp"

namespace hh {

hh_status launch_bucketed(const HashArgs& a, hipStream_t st) { return launch_quad(a, st); }

void release_bucketed() {}

}  // namespace hh
