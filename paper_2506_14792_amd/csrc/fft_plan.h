// Plan of the in-LDS mixed-radix FFT (host and device).
#pragma once

// Mixed-radix Stockham plan for length n: passes of radix 8, 6, 4, 3 or 2.  Per pass s, with
// Ns = product of the earlier radices: the divisions by n / radix and by Ns are done with
// precomputed multipliers (q = umulhi(x, mag) = floor(x / d) for x d < 2^32; mag = 0 means
// d = 1), and tst = n / (Ns radix) is the twiddle stride.
struct FftPlan {
  int n;
  int nst;
  int radix[12];
  int ns[12];
  int tst[12];
  unsigned mag_nr[12];
  unsigned mag_ns[12];
};

// LDS index padding for the FFT buffers: one spare slot after every 8 complex entries, so a
// wave writing or reading with a stride of 8 entries (128 bytes) spreads over all banks.
__host__ __device__ __forceinline__ int fpad(int i) { return i + (i >> 3); }
__host__ __device__ inline int fpad_size(int count) { return count + (count >> 3) + 1; }

namespace sps {
// Fills p for length n = 2^a 3^b (n <= 16384); false for other lengths.
bool fft_plan(int n, FftPlan* p);
}  // namespace sps
