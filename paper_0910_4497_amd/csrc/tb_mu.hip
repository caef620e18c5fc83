// Global chemical potential and the spectral sums (Sec. 2, Eq. 2: the
// occupation f of the density matrix; one mu for the whole system).
//
//   N(mu) = sum_i sum_m f(lambda_m^i) w_m^i,  f(e) = 2 / (1 + exp((e - mu)/kT)),
// solved for N(mu) = N_e. N is increasing in mu; every launch of k_mu_iter
// evaluates N at 31 points of the bracket [lo, hi] and keeps the tightest
// bracket they give. The first launch splits it into 32 equal parts; later
// launches place 24 points evenly (25 parts: 4.6 bits whatever happens) and 7
// around the root of the straight line through (lo, N(lo)) and (hi, N(hi)),
// at offsets 0, +-2^-20, +-2^-12 and +-2^-4 of the bracket width. Once the
// bracket is narrow against kT, N is nearly linear on it and the new bracket
// is the gap between two of those points (12 to 20 bits per launch): about 7
// launches reach rounding level where plain multisection takes 12, and 13
// launches cover 60 bits in any case. A fixed number
// of launches is enqueued; once the bracket has collapsed to rounding level,
// later launches return at once, so the sequence is capturable in a graph. Reductions are two-level and in a
// fixed order (per-block partials summed by the last block to finish), so
// the result is bitwise reproducible run to run.
#include <float.h>

#include "tb_internal.h"

namespace tbk {

constexpr int MU_NT = 256;
constexpr int MU_NB = 256;         // blocks of the reduction kernels (timed: 128, 256, 512)
constexpr int MU_P = 31;           // points per multisection step
constexpr int MU_U = 24;           // of which evenly spaced after the first step

enum { MS_LO = 0, MS_HI = 1, MS_MU = 2, MS_DONE = 3, MS_N = 4, MS_STEP = 5, MS_IT = 6, MS_NLO = 7, MS_NHI = 8 };


// Sum M values over the grid. Every block stores its M block sums (fixed
// order: waves, then the waves' results) in partial[block][M]; the last block
// to finish sums the blocks in a fixed tree (thread t takes blocks t, t +
// MU_NT, ..., then the wave and workgroup reductions) and returns true with
// the totals in tot[0..M-1] (shared memory of that block). OP 0 sums, OP 1
// takes minima.
template <int M, int OP>
__device__ bool grid_reduce(double (&v)[M], double* partial, unsigned int* counter, double* tot) {
  __shared__ double red[MU_NT / 64][M];
  __shared__ bool last;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  auto comb = [](double a, double b) { return OP == 0 ? a + b : fmin(a, b); };
  const double ident = OP == 0 ? 0.0 : 1e300;
#pragma unroll
  for (int q = 0; q < M; ++q)
    for (int off = 32; off > 0; off >>= 1) v[q] = comb(v[q], __shfl_xor(v[q], off, 64));
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < M; ++q) red[wave][q] = v[q];
  __syncthreads();
  if (tid < M) {
    double sm = ident;
    for (int w = 0; w < MU_NT / 64; ++w) sm = comb(sm, red[w][tid]);
    partial[(size_t)blockIdx.x * M + tid] = sm;
    __threadfence();
  }
  __syncthreads();
  if (tid == 0) last = (atomicAdd(counter, 1u) == gridDim.x - 1);
  __syncthreads();
  if (!last) return false;
  __threadfence();
  double acc[M];
#pragma unroll
  for (int q = 0; q < M; ++q) acc[q] = ident;
  for (unsigned int bk = tid; bk < gridDim.x; bk += MU_NT)
#pragma unroll
    for (int q = 0; q < M; ++q) acc[q] = comb(acc[q], partial[(size_t)bk * M + q]);
#pragma unroll
  for (int q = 0; q < M; ++q)
    for (int off = 32; off > 0; off >>= 1) acc[q] = comb(acc[q], __shfl_xor(acc[q], off, 64));
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < M; ++q) red[wave][q] = acc[q];
  __syncthreads();
  if (tid < M) {
    double sm = ident;
    for (int w = 0; w < MU_NT / 64; ++w) sm = comb(sm, red[w][tid]);
    tot[tid] = sm;
  }
  if (tid == 0) *counter = 0u;
  __syncthreads();
  return true;
}

__global__ void __launch_bounds__(MU_NT) k_mu_bracket(MuArgs g, double mu_fixed, int fixed) {
  double v[2] = {1e300, 1e300};        // min lambda, -max lambda
  for (int64_t q = (int64_t)blockIdx.x * MU_NT + threadIdx.x; q < g.n_pairs; q += (int64_t)gridDim.x * MU_NT) {
    const double l = g.lam[q];
    v[0] = fmin(v[0], l);
    v[1] = fmin(v[1], -l);
  }
  __shared__ double tot[2];
  if (grid_reduce<2, 1>(v, g.partial, g.counter, tot) && threadIdx.x == 0) {
    double* s = g.state;
    s[MS_LO] = tot[0] - 50.0 * g.kT;
    s[MS_HI] = -tot[1] + 50.0 * g.kT;
    s[MS_MU] = fixed ? mu_fixed : 0.5 * (s[MS_LO] + s[MS_HI]);
    s[MS_DONE] = fixed ? 1.0 : 0.0;
    s[MS_STEP] = s[MS_HI] - s[MS_LO];
    s[MS_IT] = 0.0;
    s[MS_NLO] = 0.0; s[MS_NHI] = 0.0;        // N at lo and hi: known after the first step
  }
}

// One multisection step: N(mu) at MU_P points of [lo, hi] (mu_point); the
// bracket becomes the tightest one among them: lo' the largest point with
// N < N_e, hi' the smallest with N >= N_e (N at a point equal to N_e exactly
// ends the search there). Sums are per block in a fixed order, then per point
// over the blocks in a fixed order by the last block, so the result is
// reproducible bit for bit.
__device__ __forceinline__ double mu_point(const double* s, double ne, int p) {
  const double lo = s[MS_LO], hi = s[MS_HI], w = hi - lo;
  if (s[MS_IT] == 0.0) return lo + (p + 1) * (w / (MU_P + 1));
  if (p < MU_U) return lo + (p + 1) * (w / (MU_U + 1));
  const double nlo = s[MS_NLO], nhi = s[MS_NHI];
  double ms = (nhi > nlo) ? lo + (ne - nlo) / (nhi - nlo) * w : 0.5 * (lo + hi);
  const int q = p - MU_U;                        // 0: the line's root; 2i-1, 2i: -+ 2^(-20+8(i-1)) w
  if (q > 0) {
    const double off = w * __builtin_amdgcn_ldexp(1.0, -20 + 8 * ((q - 1) >> 1));
    ms += (q & 1) ? -off : off;
  }
  return fmin(fmax(ms, lo), hi);
}

__global__ void __launch_bounds__(MU_NT) k_mu_iter(MuArgs g) {
  if (g.state[MS_DONE] != 0.0) return;
  const double lo = g.state[MS_LO], hi = g.state[MS_HI];
  const double cut = 40.0 * g.kT;                 // f = 0 or 2 to rounding beyond this
  double xs[MU_P];
#pragma unroll
  for (int p = 0; p < MU_P; ++p) xs[p] = mu_point(g.state, g.n_e, p);
  double v[MU_P];
#pragma unroll
  for (int p = 0; p < MU_P; ++p) v[p] = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * MU_NT + threadIdx.x; q < g.n_pairs; q += (int64_t)gridDim.x * MU_NT) {
    const double w = g.wgt[q];
    if (w == 0.0) continue;
    const double l = g.lam[q];
    if (l < lo - cut) {
#pragma unroll
      for (int p = 0; p < MU_P; ++p) v[p] += 2.0 * w;
    } else if (l <= hi + cut) {
#pragma unroll
      for (int p = 0; p < MU_P; ++p) {
        const double z = (l - xs[p]) / g.kT;
        const double e = exp(-fabs(z));
        const double f = (z > 0.0) ? 2.0 * e / (1.0 + e) : 2.0 / (1.0 + e);
        v[p] += f * w;
      }
    }
  }
  __shared__ double Np[MU_P];
  if (!grid_reduce<MU_P, 0>(v, g.partial, g.counter, Np)) return;
  const int tid = threadIdx.x;
  if (tid == 0) {
    double* s = g.state;
    double nlo = lo, nhi = hi, Nlo = s[MS_NLO], Nhi = s[MS_NHI];
    int exact = -1;
    for (int p = 0; p < MU_P; ++p) {
      if (Np[p] < g.n_e) {
        if (xs[p] > nlo) { nlo = xs[p]; Nlo = Np[p]; }
      } else {
        if (xs[p] < nhi) { nhi = xs[p]; Nhi = Np[p]; }
        if (Np[p] == g.n_e && exact < 0) exact = p;
      }
    }
    if (exact >= 0) nlo = nhi = xs[exact];
    else if (nlo >= nhi) nlo = nhi = 0.5 * (nlo + nhi);   // N not monotone at rounding level
    s[MS_LO] = nlo; s[MS_HI] = nhi; s[MS_NLO] = Nlo; s[MS_NHI] = Nhi; s[MS_IT] += 1.0;
    s[MS_MU] = 0.5 * (nlo + nhi);
    const double scale = fmax(1.0, fabs(s[MS_MU]));
    if (nhi - nlo <= 4.0 * DBL_EPSILON * scale) s[MS_DONE] = 1.0;
  }
}

// Final sums at mu: electron count, band energy, entropy S/k_B.
__global__ void __launch_bounds__(MU_NT) k_mu_final(MuArgs g) {
  const double mu = g.state[MS_MU];
  double v[3] = {0.0, 0.0, 0.0};
  for (int64_t q = (int64_t)blockIdx.x * MU_NT + threadIdx.x; q < g.n_pairs; q += (int64_t)gridDim.x * MU_NT) {
    const double w = g.wgt[q];
    const double l = g.lam[q];
    const double z = (l - mu) / g.kT;
    const double a = fabs(z);
    const double e = exp(-a);
    const double f = (z > 0.0) ? 2.0 * e / (1.0 + e) : 2.0 / (1.0 + e);
    v[0] += f * w;
    v[1] += l * f * w;
    v[2] += w * 2.0 * (log1p(e) + a * e / (1.0 + e));
  }
  __shared__ double tot[3];
  if (grid_reduce<3, 0>(v, g.partial, g.counter, tot) && threadIdx.x == 0) {
    g.eparts[0] = tot[1];      // E_band
    g.eparts[1] = tot[2];      // S / k_B
    g.eparts[3] = tot[0];      // electron count at mu
    if (g.mu_out) *g.mu_out = mu;
  }
}

int mu_blocks(int64_t n_pairs) {
  int64_t b = (n_pairs + MU_NT - 1) / MU_NT;
  if (b > MU_NB) b = MU_NB;
  if (b < 1) b = 1;
  return (int)b;
}

void launch_mu(const MuArgs& a, double mu_fixed, bool fixed, int n_iter, hipStream_t st) {
  const int nb = mu_blocks(a.n_pairs);
  hipLaunchKernelGGL(k_mu_bracket, dim3(nb), dim3(MU_NT), 0, st, a, mu_fixed, fixed ? 1 : 0);
  if (!fixed)
    for (int it = 0; it < n_iter; ++it) hipLaunchKernelGGL(k_mu_iter, dim3(nb), dim3(MU_NT), 0, st, a);
  hipLaunchKernelGGL(k_mu_final, dim3(nb), dim3(MU_NT), 0, st, a);
}

}  // namespace tbk
