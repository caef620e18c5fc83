// Global chemical potential and the spectral sums (Sec. 2, Eq. 2: the
// occupation f of the density matrix; one mu for the whole system).
//
//   N(mu) = sum_i sum_m f(lambda_m^i) w_m^i,  f(e) = 2 / (1 + exp((e - mu)/kT)),
// solved for N(mu) = N_e. N is increasing in mu; every launch of k_mu_iter
// evaluates N and dN/dmu at the current trial point over all Ritz pairs,
// tightens the bracket [lo, hi] and proposes the next point (Newton step
// when it stays inside the bracket and at least halves the previous step,
// else bisection). A fixed number of launches is enqueued; once the bracket
// has collapsed to rounding level, later launches return at once, so the
// sequence is capturable in a graph. Reductions are two-level and in a
// fixed order (per-block partials summed by the last block to finish), so
// the result is bitwise reproducible run to run.
#include <float.h>

#include "tb_internal.h"

namespace tbk {

constexpr int MU_NT = 256;
constexpr int MU_NB = 512;         // blocks of the reduction kernels

enum { MS_LO = 0, MS_HI = 1, MS_MU = 2, MS_DONE = 3, MS_N = 4, MS_STEP = 5, MS_IT = 6 };


__device__ __forceinline__ void fermi_and_deriv(double lam, double mu, double kT, double& f, double& df) {
  const double z = (lam - mu) / kT;
  const double e = exp(-fabs(z));
  f = (z > 0.0) ? 2.0 * e / (1.0 + e) : 2.0 / (1.0 + e);
  df = f * (1.0 - 0.5 * f) / kT;     // d f / d mu
}

// Block-level sum of M values into partial[blockIdx][M]; returns true in the
// last block to finish (after which partials of every block are visible).
template <int M>
__device__ bool reduce_partials(double (&v)[M], double* partial, unsigned int* counter) {
  __shared__ double red[MU_NT / 64][M];
  __shared__ bool last;
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < M; ++q) v[q] = wave_sum(v[q]);
  if ((tid & 63) == 0)
#pragma unroll
    for (int q = 0; q < M; ++q) red[tid >> 6][q] = v[q];
  __syncthreads();
  if (tid == 0) {
    for (int q = 0; q < M; ++q) {
      double s = 0.0;
      for (int w = 0; w < MU_NT / 64; ++w) s += red[w][q];
      partial[(size_t)blockIdx.x * M + q] = s;
    }
    __threadfence();
    const unsigned int t = atomicAdd(counter, 1u);
    last = (t == gridDim.x - 1);
    __threadfence();
  }
  __syncthreads();
  return last;
}

__global__ void __launch_bounds__(MU_NT) k_mu_bracket(MuArgs g, double mu_fixed, int fixed) {
  double v[2] = {1e300, 1e300};        // min lambda, -max lambda
  for (int64_t q = (int64_t)blockIdx.x * MU_NT + threadIdx.x; q < g.n_pairs; q += (int64_t)gridDim.x * MU_NT) {
    const double l = g.lam[q];
    v[0] = fmin(v[0], l);
    v[1] = fmin(v[1], -l);
  }
  __shared__ double red[MU_NT / 64][2];
  __shared__ bool last;
  const int tid = threadIdx.x;
  for (int off = 32; off > 0; off >>= 1) {
    v[0] = fmin(v[0], __shfl_xor(v[0], off, 64));
    v[1] = fmin(v[1], __shfl_xor(v[1], off, 64));
  }
  if ((tid & 63) == 0) { red[tid >> 6][0] = v[0]; red[tid >> 6][1] = v[1]; }
  __syncthreads();
  if (tid == 0) {
    double a = 1e300, b = 1e300;
    for (int w = 0; w < MU_NT / 64; ++w) { a = fmin(a, red[w][0]); b = fmin(b, red[w][1]); }
    g.partial[2 * blockIdx.x] = a;
    g.partial[2 * blockIdx.x + 1] = b;
    __threadfence();
    last = (atomicAdd(g.counter, 1u) == gridDim.x - 1);
    __threadfence();
  }
  __syncthreads();
  if (last && tid == 0) {
    double a = 1e300, b = 1e300;
    for (unsigned int w = 0; w < gridDim.x; ++w) { a = fmin(a, g.partial[2 * w]); b = fmin(b, g.partial[2 * w + 1]); }
    double* s = g.state;
    s[MS_LO] = a - 50.0 * g.kT;
    s[MS_HI] = -b + 50.0 * g.kT;
    s[MS_MU] = fixed ? mu_fixed : 0.5 * (s[MS_LO] + s[MS_HI]);
    s[MS_DONE] = fixed ? 1.0 : 0.0;
    s[MS_STEP] = s[MS_HI] - s[MS_LO];
    s[MS_IT] = 0.0;
    *g.counter = 0u;
  }
}

__global__ void __launch_bounds__(MU_NT) k_mu_iter(MuArgs g) {
  if (g.state[MS_DONE] != 0.0) return;
  const double mu = g.state[MS_MU];
  double v[2] = {0.0, 0.0};
  for (int64_t q = (int64_t)blockIdx.x * MU_NT + threadIdx.x; q < g.n_pairs; q += (int64_t)gridDim.x * MU_NT) {
    const double w = g.wgt[q];
    double f, df;
    fermi_and_deriv(g.lam[q], mu, g.kT, f, df);
    v[0] += f * w;
    v[1] += df * w;
  }
  const bool last = reduce_partials<2>(v, g.partial, g.counter);
  if (last && threadIdx.x == 0) {
    double N = 0.0, dN = 0.0;
    for (unsigned int b = 0; b < gridDim.x; ++b) { N += g.partial[2 * b]; dN += g.partial[2 * b + 1]; }
    double* s = g.state;
    double lo = s[MS_LO], hi = s[MS_HI];
    if (N < g.n_e) lo = mu; else hi = mu;
    double next = 0.5 * (lo + hi);
    if (dN > 0.0) {
      const double newton = mu - (N - g.n_e) / dN;
      if (newton > lo && newton < hi && fabs(newton - mu) < 0.5 * s[MS_STEP]) next = newton;
    }
    const double step = fabs(next - mu);
    s[MS_LO] = lo; s[MS_HI] = hi; s[MS_N] = N; s[MS_IT] += 1.0;
    const double scale = fmax(1.0, fabs(mu));
    if (N == g.n_e || step <= 4.0 * DBL_EPSILON * scale || hi - lo <= 4.0 * DBL_EPSILON * scale) {
      s[MS_DONE] = 1.0;
      if (N != g.n_e && step > 0.0) s[MS_MU] = next; else s[MS_MU] = mu;
    } else {
      s[MS_MU] = next;
      s[MS_STEP] = step;
    }
    *g.counter = 0u;
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
  const bool last = reduce_partials<3>(v, g.partial, g.counter);
  if (last && threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (unsigned int b = 0; b < gridDim.x; ++b) {
      s0 += g.partial[3 * b]; s1 += g.partial[3 * b + 1]; s2 += g.partial[3 * b + 2];
    }
    g.eparts[0] = s1;      // E_band
    g.eparts[1] = s2;      // S / k_B
    g.eparts[3] = s0;      // electron count at mu
    if (g.mu_out) *g.mu_out = mu;
    *g.counter = 0u;
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
