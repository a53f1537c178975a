// Learned gauge-covariant smoother (parallel-transport convolutions).
#pragma once
#include "lib.h"

namespace mgm {

struct Net;
// e = N(r) on the fine level (F32 vectors)
void net_apply(Hier& H, Net& net, Vec r, Vec e);

}  // namespace mgm
