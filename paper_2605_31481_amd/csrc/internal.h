// Host helpers of the C ABI shared by its translation units (not public).
#pragma once

#include <string>

#include "launch.h"
#include "status.h"

namespace bard {

// Record `msg` as the calling thread's last error and return `code`.
int fail(int code, const std::string& msg);
// BARD_E_DEVICE if an earlier asynchronous device error is pending (and clear it).
int check_device_state();
// Largest dynamic LDS allocation of one workgroup on device `dev`.
size_t lds_limit(int dev);
// True if `st` is being captured into a HIP graph (then nothing may be
// allocated or copied synchronously on its behalf).
bool capturing(hipStream_t st);
// Upload the model's tables to the current device (once per device).  On a
// first use while `st` is being captured: BARD_E_CAPTURE.
int ensure_device(bard_model* m, DeviceCopy** out, hipStream_t st);
// Device image of the Jacobian output lists for an end-effector set (cached
// per set); BARD_E_CAPTURE as for ensure_device.
int ensure_ee(bard_model* m, DeviceCopy* dc, int n_ee, const int32_t* ee_body, DevEE* out, hipStream_t st);
// Waves per workgroup for the phases after the level sweep (rs: scalar bytes).
int out_waves(int rs);

}  // namespace bard
