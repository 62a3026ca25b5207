// Request loop (placeholder until the batching server lands).
#include "sd.h"

extern "C" {
int sd_server_create(const sd_server_opts*, sd_server** out) {
  if (out) *out = nullptr;
  return SD_E_INVALID;
}
int sd_submit(sd_server*, const sd_request*, uint64_t*) { return SD_E_INVALID; }
int sd_poll(sd_server*, uint64_t, sd_result*) { return SD_E_INVALID; }
int sd_wait(sd_server*, uint64_t, double, sd_result*) { return SD_E_INVALID; }
int sd_result_release(sd_server*, uint64_t) { return SD_E_INVALID; }
int sd_cancel(sd_server*, uint64_t) { return SD_E_INVALID; }
void sd_server_destroy(sd_server*) {}
}
