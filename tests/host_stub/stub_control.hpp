// Controls of the HIP stand-in used by the host lifetime harness.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

// Make the n-th stub call of the calling thread fail (n < 1: never) and reset
// the thread's call count.
void stub_set_fail_at(long n);
// Stub calls made by the calling thread since the last stub_set_fail_at.
long stub_calls();
// Index of the call that failed by injection, or -1.
long stub_failed_at();
// Run every operation still queued on stream s (what a DMA engine would still
// complete after the caller has moved on).
void stub_drain(hipStream_t s);
size_t stub_pending(hipStream_t s);

// Sweep launches (kind 0: the iterate read and written, FP32 or not) and zero
// fills (kind 1: the buffer) of the calling thread, recorded while on.
struct StubRec {
  int kind;
  bool fp32;
  const void* in;
  const void* out;
};
void stub_record(bool on);
std::vector<StubRec> stub_records();
