#include "../../include/bires.h"

extern "C" {
int bires_server_create(size_t, int, bires_server**) { return BIRES_EINVAL; }
int bires_server_submit(bires_server*, int, int, const bires_bipoly*, const bires_bipoly*, uint64_t*) { return BIRES_EINVAL; }
int bires_server_wait(bires_server*, uint64_t, bires_upoly*, double, double*) { return BIRES_EINVAL; }
int bires_server_destroy(bires_server*) { return BIRES_EINVAL; }
}
