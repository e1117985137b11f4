// FFT-FDMT (Sec. 5, Algorithm 2): the transform with its time axis Fourier
// transformed, so that every shift becomes a product with a shift vector.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

namespace fdmt {

struct Plan;

// Longest time axis (samples after padding) an FFT plan accepts.
constexpr int64_t kFftMaxLength = int64_t(1) << 24;

// FFT length for a record of nt samples and nd delays: the smallest 2^a 3^b 5^c
// of at least nt + nd - 1 samples (the zero padding after which no path wraps).
int64_t fft_length(int64_t nt, int nd);

// Builds the plan's FFT state: shift-vector table and hipFFT plans (which
// allocate their own work areas). Returns "" on success.
std::string fft_create(Plan &p);
void fft_destroy(Plan &p);

// Workspace of one forward call (beams run one after another).
size_t fft_workspace_bytes(const Plan &p);

// Enqueues the forward transform of `batch` beams on `stream`. Returns "" on
// success, else what failed.
std::string launch_forward_fft(const Plan &p, const void *in, void *out, int batch, void *ws,
                               hipStream_t stream);

} // namespace fdmt
