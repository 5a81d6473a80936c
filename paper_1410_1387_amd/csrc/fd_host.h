// fd_host.h -- host-side helpers shared by the translation units of the C ABI
// (library-internal, hidden from the exported symbol table).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdw {

// Records a printf-style message as the calling thread's last error and returns code.
__attribute__((visibility("hidden"), format(printf, 2, 3))) int host_fail(int code, const char *fmt, ...);

// Workgroups of `kernel` (nt threads) the whole device runs at once.
__attribute__((visibility("hidden"))) int resident_slots(const void *kernel, int nt);

// Planes per z chunk for tiles_xy tiles over nz planes with a z halo of r planes.
__attribute__((visibility("hidden"))) int choose_zch(int64_t tiles_xy, int64_t nz, int r, int slots);

}  // namespace fdw
