// Library-internal entry points shared between translation units (not part
// of the C ABI).
#pragma once

#include <cstddef>
#include <cstdint>

#include "../../include/esp.h"

namespace espx {

// esp_plan with every device buffer carved out of the caller's region
// [base, base + cap) (no device allocation; ESP_ENOMEM with a message when the
// plan does not fit).  Such a plan serves esp_forces only (it holds no
// real-space buffers) and does not free the region.  Buffers that must start
// at zero are cleared by fill kernels on o->stream.
esp_status plan_in_region(const double h[9], int64_t n, double tol, const esp_opts* o, void* base, size_t cap,
                          esp_plan_t** out, size_t* used);

// Frees the host side of a plan without synchronising its stream (work it
// enqueued keeps running; a region plan's device memory is the caller's).
void plan_release(esp_plan_t* p);

// True when esp_plan, given the cell h and the plan's own n, tol and options,
// would choose the grid and tiles the plan already has, so that esp_set_box(h)
// makes it the plan esp_plan would make (analytic and explicit parameters).
bool plan_same_grid(const esp_plan_t* p, const double h[9]);

}  // namespace espx
