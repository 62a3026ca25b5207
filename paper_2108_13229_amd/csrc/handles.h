// Handle types of the C ABI shared by the translation units that implement it.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "sd.h"
#include "sd_internal.h"

struct sd_problem {
  sd::HostProblem hp;
  bool device = false;
  int device_id = 0;
  sd_allocator alloc{};
  bool has_alloc = false;
  hipStream_t stream = nullptr;
};

namespace sd {

// Records the thread-local message returned by sd_last_error().
void set_last_error(const std::string& msg);

// Runs f, turning exceptions into sd_status codes and messages.
template <typename F>
int guarded_call(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return SD_E_NOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return SD_E_INVALID;
  } catch (...) {
    set_last_error("unknown error");
    return SD_E_INVALID;
  }
}

}  // namespace sd
