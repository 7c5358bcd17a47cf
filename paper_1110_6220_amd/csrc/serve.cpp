// Serving entry points (continuous batching).  See include/eik.h.
#include <cstring>
#include <string>

#include "../../include/eik.h"

extern "C" {

int eik_serve_create(const eik_serve_cfg*, eik_server** out) {
  if (out) *out = nullptr;
  return EIK_EINVAL;
}
int eik_serve_submit(eik_server*, const eik_problem*, uint64_t*) { return EIK_EINVAL; }
int eik_serve_poll(eik_server*, uint64_t, eik_stats*) { return EIK_EINVAL; }
int eik_serve_wait(eik_server*, uint64_t, eik_stats*) { return EIK_EINVAL; }
int eik_serve_cancel(eik_server*, uint64_t) { return EIK_EINVAL; }
int eik_serve_destroy(eik_server*) { return EIK_EINVAL; }

}  // extern "C"
