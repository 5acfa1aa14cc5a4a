// Precision dispatch of the kernel launchers: the kernels exist once per
// working precision (namespaces sgn::p64 and sgn::p32, compiled from the same
// source); Geom::fp32 selects the set.
#include "sgn_launch.hpp"

namespace sgn {

thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;
thread_local unsigned t_members = 1;

void set_launch_events(hipEvent_t start, hipEvent_t stop) {
  t_ev_start = start;
  t_ev_stop = stop;
}

#define SGN_DEFINE_DISPATCH(name, params, args)                                        \
  hipError_t launch_##name params {                                                   \
    t_members = g.members > 1 ? (unsigned)g.members : 1u;                             \
    const hipError_t e = g.fp32 ? p32::launch_##name args : p64::launch_##name args; \
    t_members = 1;                                                                    \
    return e;                                                                         \
  }
SGN_LAUNCHERS(SGN_DEFINE_DISPATCH)

int max_partial_blocks(const Geom& g) { return g.fp32 ? p32::max_partial_blocks(g) : p64::max_partial_blocks(g); }
bool chained_ok(const Geom& g) { return g.fp32 ? p32::chained_ok(g) : p64::chained_ok(g); }
void launch_shape(const Geom& g, int* out4) { g.fp32 ? p32::launch_shape(g, out4) : p64::launch_shape(g, out4); }

}  // namespace sgn
