// FFT-FDMT (Sec. 5, Algorithm 2). The Option-1 rows of every channel are
// built in the time domain, zero-padded to n >= Nt + Nd - 1 samples and
// Fourier transformed along time (hipFFT, real to complex). Each iteration
// then adds, at every frequency bin w of the time axis,
//   B_out(w) = B_lo(w) + B_hi(w) * V(w, s),  V(w, s) = exp(-2 pi i w s / n),
// the transform of a unit impulse at s, so all additions stay within one bin.
// Iterations run kFftLevels at a time: an output row of plane l1 is the sum of
// its 2^k terms of plane l0 (the rows the recursion reaches, each with its
// accumulated shift sigma), each times V(w, sigma), which is the recursion
// with its shifts composed (V(w, a) V(w, b) = V(w, a + b)).
// The last plane is transformed back (complex to real), scaled by 1/n and cut
// to the record. The padding makes the cyclic shifts of the transform equal
// the zero-history shifts of the direct algorithm: a path reads samples in
// [t0 - dt, t0], dt <= Nd - 1, so a wrapped read lands in the zero tail.
//
// Layout: plane rows of rpitch reals (time) or cpitch complex bins
// (frequency), both multiples of 64 elements; beams run one after another
// through the same buffers.
#include "fdmt_fft.h"

#include <hipfft/hipfft.h>

#include <cmath>
#include <vector>

#include "fdmt_plan.h"

namespace fdmt {

struct FftPlan {
  struct Pass {
    int l0, l1;           // consumes plane l0, produces plane l1
    int64_t term_offset;  // first (row, shift) term of this pass, 2^(l1-l0) per output row
  };
  int64_t n = 0;        // FFT length: the record plus its zero padding
  int64_t rpitch = 0;   // reals per time-domain row
  int64_t nbins = 0;    // n / 2 + 1 complex bins of a real row's transform
  int64_t cpitch = 0;   // complex elements per frequency-domain row
  int64_t rows0 = 0;    // rows of plane 0 (Option-1 rows of every channel position)
  hipfftHandle r2c = nullptr, c2r = nullptr;
  float2 *twiddle = nullptr;  // V(1, k) = exp(-2 pi i k / n), k < n
  int2 *terms = nullptr;      // every pass's terms
  std::vector<Pass> passes;
};

namespace {

constexpr int kFftThreads = 256;
constexpr int kBinsPerThread = 4;
constexpr int kFftLevels = 3;  // iterations per frequency-domain pass

const char *fft_error(hipfftResult r) {
  switch (r) {
    case HIPFFT_SUCCESS: return "";
    case HIPFFT_ALLOC_FAILED: return "hipFFT allocation failed";
    case HIPFFT_INVALID_VALUE: return "hipFFT invalid value";
    case HIPFFT_INVALID_SIZE: return "hipFFT invalid size";
    case HIPFFT_EXEC_FAILED: return "hipFFT execution failed";
    default: return "hipFFT error";
  }
}

// Zeros samples from..pitch-1 of every row: the padding after the record.
__global__ __launch_bounds__(kFftThreads) void pad_tail_kernel(float *__restrict__ base, int64_t pitch,
                                                               int64_t from) {
  float *row = base + static_cast<int64_t>(blockIdx.x) * pitch;
  for (int64_t t = from + threadIdx.x; t < pitch; t += kFftThreads) row[t] = 0.0f;
}

// k iterations in the frequency domain. Grid: (row of plane l1, bin tile).
// A thread takes kBinsPerThread consecutive bins w0 .. w0+3. For each term it
// looks up V(w0, sigma) once (index w0 * sigma mod n, through a float64
// quotient corrected by one step) and reaches the next bins by multiplying
// with V(1, sigma), the same for every thread: one scattered table read per
// term instead of four.
template <int K>
__global__ __launch_bounds__(kFftThreads) void fft_gather_kernel(const float2 *__restrict__ prev,
                                                                 float2 *__restrict__ next,
                                                                 const int2 *__restrict__ terms,
                                                                 const float2 *__restrict__ tw, int64_t n,
                                                                 double inv_n, int64_t cpitch, int64_t nbins) {
  constexpr int N = 1 << K;
  const int64_t r = blockIdx.x;
  const int64_t w0 = (static_cast<int64_t>(blockIdx.y) * kFftThreads + threadIdx.x) * kBinsPerThread;
  if (w0 >= nbins) return;
  const int2 *tm = terms + r * N;
  float2 acc[kBinsPerThread];
#pragma unroll
  for (int q = 0; q < kBinsPerThread; ++q) acc[q] = make_float2(0.0f, 0.0f);
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const int2 e = tm[j];  // {plane-l0 row, accumulated shift}
    // the row pitch is a multiple of 64 bins, so all four bins lie in the row
    const float4 *src = reinterpret_cast<const float4 *>(prev + e.x * cpitch + w0);
    const float4 b0 = src[0], b1 = src[1];
    const float2 bv[4] = {{b0.x, b0.y}, {b0.z, b0.w}, {b1.x, b1.y}, {b1.z, b1.w}};
    const int64_t s = e.y;
    const int64_t x = w0 * s;
    int64_t k = x - static_cast<int64_t>(static_cast<double>(x) * inv_n) * n;
    if (k < 0) k += n;
    if (k >= n) k -= n;
    float2 v = tw[k];
    const float2 step = tw[s];
#pragma unroll
    for (int q = 0; q < kBinsPerThread; ++q) {
      acc[q].x += bv[q].x * v.x - bv[q].y * v.y;
      acc[q].y += bv[q].x * v.y + bv[q].y * v.x;
      v = make_float2(v.x * step.x - v.y * step.y, v.x * step.y + v.y * step.x);
    }
  }
  float4 *out = reinterpret_cast<float4 *>(next + r * cpitch + w0);
  out[0] = make_float4(acc[0].x, acc[0].y, acc[1].x, acc[1].y);
  out[1] = make_float4(acc[2].x, acc[2].y, acc[3].x, acc[3].y);
}

// out[r][t] = real[r][t] / n for t < nt (the inverse transform is unscaled).
__global__ __launch_bounds__(kFftThreads) void fft_output_kernel(const float *__restrict__ real,
                                                                 float *__restrict__ out, int64_t rpitch,
                                                                 int64_t nt, int32_t nd, float scale) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kFftThreads + threadIdx.x;
  if (t >= nt) return;
  for (int32_t r = blockIdx.y; r < nd; r += gridDim.y) out[r * nt + t] = real[r * rpitch + t] * scale;
}

}  // namespace

int64_t fft_length(int64_t nt, int nd) {
  const int64_t need = nt + nd - 1;
  int64_t best = INT64_MAX;
  for (int64_t a = 1; a <= 2 * need; a *= 2)
    for (int64_t b = a; b <= 2 * need; b *= 3)
      for (int64_t c = b; c <= 2 * need; c *= 5)
        if (c >= need && c < best) best = c;
  return best;
}

std::string fft_create(Plan &p) {
  const Tables &T = p.tab;
  auto *f = new FftPlan;
  p.fft = f;
  f->n = fft_length(p.nt, T.nd);
  if (f->n > kFftMaxLength) return "FFT length above 2^24 samples";
  f->rpitch = round_up(f->n, kRowAlign);
  f->nbins = f->n / 2 + 1;
  f->cpitch = round_up(f->nbins, kRowAlign);
  f->rows0 = T.total[0];
  std::vector<float2> tw(f->n);
  for (int64_t k = 0; k < f->n; ++k) {
    const double a = 2.0 * M_PI * static_cast<double>(k) / static_cast<double>(f->n);
    tw[k] = make_float2(static_cast<float>(std::cos(a)), static_cast<float>(-std::sin(a)));
  }
  hipError_t e = hipMalloc(&f->twiddle, tw.size() * sizeof(float2));
  if (e != hipSuccess) {
    f->twiddle = nullptr;
    return std::string("hipMalloc of the shift-vector table: ") + hipGetErrorString(e);
  }
  e = hipMemcpy(f->twiddle, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice);
  if (e != hipSuccess) return std::string("hipMemcpy of the shift-vector table: ") + hipGetErrorString(e);
  int n = static_cast<int>(f->n), rp = static_cast<int>(f->rpitch), cp = static_cast<int>(f->cpitch);
  hipfftResult r = hipfftPlanMany(&f->r2c, 1, &n, &rp, 1, rp, &cp, 1, cp, HIPFFT_R2C, static_cast<int>(f->rows0));
  if (r != HIPFFT_SUCCESS) {
    f->r2c = nullptr;
    return std::string("forward FFT plan: ") + fft_error(r);
  }
  r = hipfftPlanMany(&f->c2r, 1, &n, &cp, 1, cp, &rp, 1, rp, HIPFFT_C2R, T.nd);
  if (r != HIPFFT_SUCCESS) {
    f->c2r = nullptr;
    return std::string("inverse FFT plan: ") + fft_error(r);
  }
  // Terms of each pass: walking the merge rows down from every output row of
  // plane l1 to plane l0, the upper half of each merge adding its shift.
  std::vector<int2> terms, cur, nxt;
  for (int l0 = 0; l0 < T.levels; l0 += kFftLevels) {
    const int l1 = std::min(l0 + kFftLevels, T.levels);
    f->passes.push_back({l0, l1, static_cast<int64_t>(terms.size())});
    for (int64_t row = 0; row < T.total[l1]; ++row) {
      cur.assign(1, make_int2(static_cast<int>(row), 0));
      for (int l = l1; l > l0; --l) {
        nxt.clear();
        for (const int2 &x : cur) {
          const MergeRow &m = T.merge[l][x.x];
          nxt.push_back(make_int2(m.lo, x.y));
          nxt.push_back(make_int2(m.hi, x.y + m.s));
        }
        cur.swap(nxt);
      }
      for (const int2 &x : cur)
        if (x.x < 0 || x.x >= T.total[l0] || x.y < 0 || x.y >= f->n) return "frequency-domain term out of range";
      terms.insert(terms.end(), cur.begin(), cur.end());
    }
  }
  if (!terms.empty()) {
    e = hipMalloc(&f->terms, terms.size() * sizeof(int2));
    if (e != hipSuccess) {
      f->terms = nullptr;
      return std::string("hipMalloc of the frequency-domain terms: ") + hipGetErrorString(e);
    }
    e = hipMemcpy(f->terms, terms.data(), terms.size() * sizeof(int2), hipMemcpyHostToDevice);
    if (e != hipSuccess) return std::string("hipMemcpy of the frequency-domain terms: ") + hipGetErrorString(e);
  }
  return "";
}

void fft_destroy(Plan &p) {
  FftPlan *f = p.fft;
  if (!f) return;
  if (f->r2c) hipfftDestroy(f->r2c);
  if (f->c2r) hipfftDestroy(f->c2r);
  if (f->twiddle) (void)hipFree(f->twiddle);
  if (f->terms) (void)hipFree(f->terms);
  delete f;
  p.fft = nullptr;
}

size_t fft_workspace_bytes(const Plan &p) {
  const FftPlan *f = p.fft;
  if (!f) return 0;
  const int64_t real_rows = std::max<int64_t>(f->rows0, p.tab.nd);
  // one time-domain plane, two frequency-domain planes
  return static_cast<size_t>(real_rows * f->rpitch) * sizeof(float) +
         2 * static_cast<size_t>(p.rmax * f->cpitch) * sizeof(float2);
}

std::string launch_forward_fft(const Plan &p, const void *in, void *out, int batch, void *ws,
                               hipStream_t stream) {
  const FftPlan *f = p.fft;
  const Tables &T = p.tab;
  const int64_t real_rows = std::max<int64_t>(f->rows0, T.nd);
  float *real = static_cast<float *>(ws);
  float2 *spec[2] = {reinterpret_cast<float2 *>(real + real_rows * f->rpitch), nullptr};
  spec[1] = spec[0] + p.rmax * f->cpitch;
  if (hipfftSetStream(f->r2c, stream) != HIPFFT_SUCCESS || hipfftSetStream(f->c2r, stream) != HIPFFT_SUCCESS)
    return "hipfftSetStream failed";
  const size_t in_b = p.in_dtype == FDMT_U8 ? 1 : (p.in_dtype == FDMT_F16 ? 2 : 4);
  const unsigned bin_tiles = static_cast<unsigned>((f->nbins + kFftThreads * kBinsPerThread - 1) /
                                                   (kFftThreads * kBinsPerThread));
  for (int b = 0; b < batch; ++b) {
    const void *x = static_cast<const unsigned char *>(in) + static_cast<size_t>(b) * T.nf * p.nt * in_b;
    float *y = static_cast<float *>(out) + static_cast<size_t>(b) * T.nd * p.nt;
    // Option-1 rows in the time domain, then the zero tail
    hipError_t e = launch_init_f32(p, x, real, f->rpitch, stream);
    if (e != hipSuccess) return std::string("initialisation: ") + hipGetErrorString(e);
    if (f->rpitch > p.nt) {
      hipLaunchKernelGGL(pad_tail_kernel, dim3(static_cast<unsigned>(f->rows0)), dim3(kFftThreads), 0, stream, real,
                         f->rpitch, p.nt);
      e = hipGetLastError();
      if (e != hipSuccess) return std::string("padding: ") + hipGetErrorString(e);
    }
    hipfftResult r = hipfftExecR2C(f->r2c, real, reinterpret_cast<hipfftComplex *>(spec[0]));
    if (r != HIPFFT_SUCCESS) return std::string("forward FFT: ") + fft_error(r);
    const double inv_n = 1.0 / static_cast<double>(f->n);
    int cur = 0;
    for (const FftPlan::Pass &ps : f->passes) {
      const dim3 grid(static_cast<unsigned>(T.total[ps.l1]), bin_tiles);
      const int2 *tm = f->terms + ps.term_offset;
      switch (ps.l1 - ps.l0) {
        case 1:
          hipLaunchKernelGGL(fft_gather_kernel<1>, grid, dim3(kFftThreads), 0, stream, spec[cur], spec[cur ^ 1], tm,
                             f->twiddle, f->n, inv_n, f->cpitch, f->nbins);
          break;
        case 2:
          hipLaunchKernelGGL(fft_gather_kernel<2>, grid, dim3(kFftThreads), 0, stream, spec[cur], spec[cur ^ 1], tm,
                             f->twiddle, f->n, inv_n, f->cpitch, f->nbins);
          break;
        default:
          hipLaunchKernelGGL(fft_gather_kernel<kFftLevels>, grid, dim3(kFftThreads), 0, stream, spec[cur],
                             spec[cur ^ 1], tm, f->twiddle, f->n, inv_n, f->cpitch, f->nbins);
          break;
      }
      e = hipGetLastError();
      if (e != hipSuccess) return std::string("frequency-domain pass: ") + hipGetErrorString(e);
      cur ^= 1;
    }
    r = hipfftExecC2R(f->c2r, reinterpret_cast<hipfftComplex *>(spec[cur]), real);
    if (r != HIPFFT_SUCCESS) return std::string("inverse FFT: ") + fft_error(r);
    const unsigned gx = static_cast<unsigned>((p.nt + kFftThreads - 1) / kFftThreads);
    const unsigned gy = static_cast<unsigned>(std::min<int64_t>(T.nd, 65535));
    hipLaunchKernelGGL(fft_output_kernel, dim3(gx, gy), dim3(kFftThreads), 0, stream, real, y, f->rpitch, p.nt, T.nd,
                       static_cast<float>(1.0 / static_cast<double>(f->n)));
    e = hipGetLastError();
    if (e != hipSuccess) return std::string("output: ") + hipGetErrorString(e);
  }
  return "";
}

} // namespace fdmt
