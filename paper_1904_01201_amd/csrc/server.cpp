// Serving loop (continuous batching over resident scenes).
#include "runtime.h"

extern "C" {
hab_status hab_server_create(hab_context *, const hab_server_cfg *, hab_server **) { return HAB_ERR_INVALID_ARG; }
hab_status hab_server_submit(hab_server *, const hab_view *, uint64_t *) { return HAB_ERR_INVALID_ARG; }
hab_status hab_server_poll(hab_server *, uint64_t, hab_request_stats *) { return HAB_ERR_INVALID_ARG; }
hab_status hab_server_wait(hab_server *, uint64_t, hab_request_stats *) { return HAB_ERR_INVALID_ARG; }
hab_status hab_server_stats_get(hab_server *, hab_server_stats *) { return HAB_ERR_INVALID_ARG; }
hab_status hab_server_destroy(hab_server *) { return HAB_ERR_INVALID_ARG; }
}
