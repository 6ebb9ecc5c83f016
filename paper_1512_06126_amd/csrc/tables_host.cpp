// placeholder, replaced below
#include "handle.h"
namespace giem {
int compute_tables_host(giem_handle *t, double freq, std::vector<cd> &spatial) {
  (void)t; (void)freq; (void)spatial;
  set_error("giem_tables: coefficient computation not available in this build");
  return GIEM_EINVAL;
}
}
