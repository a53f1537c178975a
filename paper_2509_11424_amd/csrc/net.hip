#include "net.h"

namespace mgm {

struct Net {
  int dummy;
};

void net_apply(Hier&, Net&, Vec, Vec) { throw Error(MGM_ERR_INVALID_ARG, "network smoother not available"); }

}  // namespace mgm
