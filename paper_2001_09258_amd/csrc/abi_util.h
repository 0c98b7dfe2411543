// Shared by the translation units of the C ABI: the calling thread's last
// error message (returned by libm_hip_last_error).
#pragma once

namespace lmh_abi {
extern thread_local char g_last_error[256];
void set_error(const char* msg);
}  // namespace lmh_abi
