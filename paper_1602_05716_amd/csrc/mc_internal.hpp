// mc_internal.hpp -- what one translation unit of the library needs from
// another (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

struct mc_handle;

// Device view of a chain's training log and the chain's stream.
struct MCLogView {
    const uint32_t* feat;   // [cap][64] packed byte histograms
    const double* de;       // [cap] exact dE
    const uint8_t* flags;   // [cap]
    int64_t cap;
    double lB;
    hipStream_t stream;
};

// Synchronises the handle and fills *out; MC_E_ARG if the chain has no log.
int mc_internal_log(mc_handle* h, int32_t chain, MCLogView* out);

// Records an error on the handle (as every entry point does) and returns code.
int mc_internal_fail(mc_handle* h, int code, const char* msg);

// Records the reason a handle-free call failed, for mc_last_error(NULL).
void mc_internal_note_error(const char* msg);
