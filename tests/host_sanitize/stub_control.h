// Controls and counters of the stub runtime (test infrastructure only).
#pragma once
#include <stddef.h>
#include <stdint.h>

// Make every stub hipMalloc of at least `bytes` fail (-1: none).
void stub_fail_allocations_of_at_least(int64_t bytes);
// Bytes of stub "device" memory allocated now, and at most since the last reset.
size_t stub_device_bytes();
size_t stub_device_peak();
void stub_reset_peak();
