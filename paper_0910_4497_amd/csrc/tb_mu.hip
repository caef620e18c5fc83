// Global chemical potential and the spectral sums (Sec. 2, Eq. 2: the
// occupation f of the density matrix; one mu for the whole system).
//
//   N(mu) = sum_i sum_m f(lambda_m^i) w_m^i,  f(e) = 2 / (1 + exp((e - mu)/kT)),
// solved for N(mu) = N_e. N is increasing in mu; every multisection step
// evaluates N at 31 points of the bracket [lo, hi] and keeps the tightest
// bracket they give. The first step splits it into 32 equal parts; later
// steps place 24 points evenly (25 parts: 4.6 bits whatever happens) and 7
// around the root of the straight line through (lo, N(lo)) and (hi, N(hi)),
// at offsets 0, +-2^-20, +-2^-12 and +-2^-4 of the bracket width. Once the
// bracket is narrow against kT, N is nearly linear on it and the new bracket
// is the gap between two of those points (12 to 20 bits per step): about 7
// steps reach rounding level where plain multisection takes 12, and 13 steps
// cover 60 bits in any case.
//
// Workgroups exchange data only across kernel boundaries. Launch q writes
// its per-block partial sums to one of two partial buffers; launch q + 1
// reads them, and every one of its blocks reduces them in the same fixed
// order (thread t takes block t, then the wave and workgroup reductions),
// so all blocks hold the same totals bit for bit and update the same bracket
// (block 0 also stores it, in the other of two state buffers, for launch
// q + 2 to read). No block reads what another block of the same launch
// writes: no tickets, counters or fences are involved, and the result is
// bitwise reproducible run to run. A fixed number of launches is enqueued;
// once the bracket has collapsed to rounding level later launches return at
// once, so the sequence is capturable in a graph.
#include <float.h>

#include "tb_internal.h"

namespace tbk {

constexpr int MU_NT = 256;
constexpr int MU_NB = 256;         // blocks of the reduction kernels (timed: 128, 256, 512)
constexpr int MU_P = 31;           // points per multisection step
constexpr int MU_U = 24;           // of which evenly spaced after the first step
constexpr int MU_PS = 32;          // partial-buffer stride per block (doubles)
static_assert(MU_NB <= MU_NT, "one block's partials per reducing thread");

// State buffer (16 doubles each; two alternate between launches).
enum { MS_LO = 0, MS_HI = 1, MS_DONE = 3, MS_IT = 6, MS_NLO = 7, MS_NHI = 8 };
// Slots of the mu_state array: two state buffers behind the final mu.
constexpr int MU_FINAL = 2;        // the chemical potential the density matrix uses
constexpr int MU_STATE0 = 16;      // state buffers at 16 and 32

// 1/q: the hardware reciprocal refined by one Newton step.
__device__ __forceinline__ double rcp_nr(double q) {
  const double r = __builtin_amdgcn_rcp(q);
  return fma(r, fma(-q, r, 1.0), r);
}

// Sums of the MU_P point values over a wave by a reduce-scatter: at each of
// the five halvings a lane keeps one half of its values and adds its
// partner's copy of that half (16 + 8 + 4 + 2 + 1 shuffles), then a last
// exchange with the neighbouring lane; lane l ends with the wave's total of
// value l / 2 (l even and odd alike).
__device__ __forceinline__ double wave_sum_points(const double (&v)[MU_P], int lane) {
  double a[32];
#pragma unroll
  for (int q = 0; q < 32; ++q) a[q] = q < MU_P ? v[q] : 0.0;
#pragma unroll
  for (int h = 16, off = 32; h >= 1; h >>= 1, off >>= 1) {
    const bool upper = (lane & off) != 0;
#pragma unroll
    for (int i = 0; i < h; ++i) {
      const double keep = upper ? a[i + h] : a[i], send = upper ? a[i] : a[i + h];
      a[i] = keep + __shfl_xor(send, off, 64);
    }
  }
  return a[0] + __shfl_xor(a[0], 1, 64);
}

// Per-block sums of M values over the workgroup (waves in order, then the
// waves' results): the totals land in out[0..M-1] (shared memory).
template <int M, int OP>
__device__ void block_reduce(double (&v)[M], double* out) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if constexpr (M == MU_P && OP == 0) {
    __shared__ double redp[MU_NT / 64][32];
    const double t = wave_sum_points(v, lane);
    if ((lane & 1) == 0) redp[wave][lane >> 1] = t;
    __syncthreads();
    if (tid < M) {
      double sm = 0.0;
      for (int w = 0; w < MU_NT / 64; ++w) sm += redp[w][tid];
      out[tid] = sm;
    }
    __syncthreads();
    return;
  }
  __shared__ double red[MU_NT / 64][M];
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
    out[tid] = sm;
  }
  __syncthreads();
}

// This block's M sums to partial[block][0..M-1].
template <int M, int OP>
__device__ void store_partials(double (&v)[M], double* partial) {
  __shared__ double tot[M];
  block_reduce<M, OP>(v, tot);
  if (threadIdx.x < M) partial[(size_t)blockIdx.x * MU_PS + threadIdx.x] = tot[threadIdx.x];
}

// Totals over the nb blocks of the previous launch: thread t takes block t,
// then the wave and workgroup reductions (the same order in every block).
template <int M, int OP>
__device__ void reduce_partials(const double* partial, int nb, double* out) {
  double acc[M];
#pragma unroll
  for (int q = 0; q < M; ++q) acc[q] = OP == 0 ? 0.0 : 1e300;
  if ((int)threadIdx.x < nb) {
    const double* src = partial + (size_t)threadIdx.x * MU_PS;
#pragma unroll
    for (int q = 0; q < M; ++q) acc[q] = src[q];
  }
  block_reduce<M, OP>(acc, out);
}

// The MU_P points of a multisection step on the bracket held in s.
__device__ __forceinline__ void mu_points(const double* s, double ne, double (&xs)[MU_P]) {
  const double lo = s[MS_LO], hi = s[MS_HI], w = hi - lo;
  if (s[MS_IT] == 0.0) {
#pragma unroll
    for (int p = 0; p < MU_P; ++p) xs[p] = lo + (p + 1) * (w / (MU_P + 1));
    return;
  }
#pragma unroll
  for (int p = 0; p < MU_U; ++p) xs[p] = lo + (p + 1) * (w / (MU_U + 1));
  const double nlo = s[MS_NLO], nhi = s[MS_NHI];
  const double ms0 = (nhi > nlo) ? lo + (ne - nlo) / (nhi - nlo) * w : 0.5 * (lo + hi);
#pragma unroll
  for (int q = 0; q < MU_P - MU_U; ++q) {        // 0: the line's root; 2i-1, 2i: -+ 2^(-20+8(i-1)) w
    double ms = ms0;
    if (q > 0) {
      const double off = w * __builtin_amdgcn_ldexp(1.0, -20 + 8 * ((q - 1) >> 1));
      ms += (q & 1) ? -off : off;
    }
    xs[MU_U + q] = fmin(fmax(ms, lo), hi);
  }
}

// The bracket after a step that evaluated N at the points of s (Np[p]):
// lo' the largest point with N < N_e, hi' the smallest with N >= N_e (N at a
// point equal to N_e exactly ends the search there). Written to t.
__device__ void mu_update(const double* s, const double* Np, double ne, double* t) {
  const double lo = s[MS_LO], hi = s[MS_HI];
  double nlo = lo, nhi = hi, Nlo = s[MS_NLO], Nhi = s[MS_NHI];
  double xs[MU_P];
  mu_points(s, ne, xs);
  int exact = -1;
#pragma unroll
  for (int p = 0; p < MU_P; ++p) {
    const double x = xs[p];
    if (Np[p] < ne) {
      if (x > nlo) { nlo = x; Nlo = Np[p]; }
    } else {
      if (x < nhi) { nhi = x; Nhi = Np[p]; }
      if (Np[p] == ne && exact < 0) exact = p;
    }
  }
  double x_exact = 0.0;
#pragma unroll
  for (int p = 0; p < MU_P; ++p) x_exact = p == exact ? xs[p] : x_exact;
  if (exact >= 0) nlo = nhi = x_exact;
  else if (nlo >= nhi) nlo = nhi = 0.5 * (nlo + nhi);   // N not monotone at rounding level
  t[MS_LO] = nlo; t[MS_HI] = nhi; t[MS_NLO] = Nlo; t[MS_NHI] = Nhi; t[MS_IT] = s[MS_IT] + 1.0;
  const double mid = 0.5 * (nlo + nhi);
  const double scale = fmax(1.0, fabs(mid));
  t[MS_DONE] = (nhi - nlo <= 4.0 * DBL_EPSILON * scale) ? 1.0 : 0.0;
}

// Per-block minimum and maximum of the Ritz values.
__global__ void __launch_bounds__(MU_NT) k_mu_bracket(MuArgs g) {
  double v[2] = {1e300, 1e300};        // min lambda, -max lambda
  for (int64_t q = (int64_t)blockIdx.x * MU_NT + threadIdx.x; q < g.n_pairs; q += (int64_t)gridDim.x * MU_NT) {
    const double l = g.lam[q];
    v[0] = fmin(v[0], l);
    v[1] = fmin(v[1], -l);
  }
  store_partials<2, 1>(v, g.partial);
}

// Adds f(x_p) w for the NE evenly spaced points x_p (E_p = exp((l - x_p)/kT)
// by products from E_0 = exp(z0), or one exponential per point when |z0| is
// beyond 600; f = 2 / (1 + E) by the refined hardware reciprocal, E kept
// below 1e300 so that 1 + E stays finite).
template <int NE>
__device__ __forceinline__ void even_points(double (&v)[MU_P], const double (&xs)[MU_P], double l, double z0,
                                            double qstep, double ikT, double w) {
  if (fabs(z0) <= 600.0) {
    double E = exp(z0);
#pragma unroll
    for (int p = 0; p < NE; ++p) {
      if (p > 0) E *= qstep;
      v[p] += 2.0 * rcp_nr(1.0 + E) * w;
    }
  } else {
#pragma unroll
    for (int p = 0; p < NE; ++p) v[p] += 2.0 * rcp_nr(1.0 + fmin(exp((l - xs[p]) * ikT), 1e300)) * w;
  }
}

// Multisection launch `it` (0-based). The bracket of this launch's points is
// that of the previous state updated with the previous launch's partials
// (it = 0: the bracket [min lambda - 50 kT, max lambda + 50 kT] from the
// extremes of k_mu_bracket). Reads partial buffer it & 1 and state buffer
// it & 1; writes partial buffer (it + 1) & 1 and (block 0) state buffer
// (it + 1) & 1.
__global__ void __launch_bounds__(MU_NT) k_mu_iter(MuArgs g, int it) {
  const double* s_in = g.state + MU_STATE0 + 16 * (it & 1);
  double* s_out = g.state + MU_STATE0 + 16 * ((it + 1) & 1);
  const double* p_in = g.partial + (size_t)(it & 1) * MU_NB * MU_PS;
  double* p_out = g.partial + (size_t)((it + 1) & 1) * MU_NB * MU_PS;
  const int nb = gridDim.x;
  __shared__ double st[16];
  __shared__ double Np[MU_P];
  if (it == 0) {
    __shared__ double ext[2];
    reduce_partials<2, 1>(g.partial, nb, ext);
    if (threadIdx.x == 0) {
      for (int q = 0; q < 16; ++q) st[q] = 0.0;
      st[MS_LO] = ext[0] - 50.0 * g.kT;
      st[MS_HI] = -ext[1] + 50.0 * g.kT;
    }
    __syncthreads();
  } else {
    if (s_in[MS_DONE] != 0.0) {                  // converged: carry the state forward
      if (blockIdx.x == 0 && threadIdx.x < 16) s_out[threadIdx.x] = s_in[threadIdx.x];
      return;
    }
    reduce_partials<MU_P, 0>(p_in, nb, Np);
    if (threadIdx.x == 0) {
      double s[16];
      for (int q = 0; q < 16; ++q) s[q] = s_in[q];
      double t[16];
      for (int q = 0; q < 16; ++q) t[q] = s[q];
      mu_update(s, Np, g.n_e, t);
      for (int q = 0; q < 16; ++q) st[q] = t[q];
    }
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x < 16) s_out[threadIdx.x] = st[threadIdx.x];
  if (st[MS_DONE] != 0.0) return;
  const double lo = st[MS_LO], hi = st[MS_HI];
  const double cut = 40.0 * g.kT;                 // f = 0 or 2 to rounding beyond this
  const double ikT = 1.0 / g.kT;
  double xs[MU_P];
  mu_points(st, g.n_e, xs);
  // f(x_p) = 2 / (1 + E_p), E_p = exp((l - x_p) / kT). The evenly spaced
  // points x_p = lo + (p + 1) h give E_{p+1} = E_p exp(-h / kT): one
  // exponential per Ritz value and a product per point. The points about the
  // line's root, x = m -+ o_i (when not clamped to the bracket), give
  // E = E_m exp(+-o_i / kT). The products add a few ulp of relative error to
  // E, far below what decides a bracket. A Ritz value more than 600 kT from
  // the first point or the root takes one exponential per point instead, so
  // no product starts from an overflowed or underflowed value.
  const bool first = st[MS_IT] == 0.0;
  const double h = first ? (hi - lo) / (MU_P + 1) : (hi - lo) / (MU_U + 1);
  const double qstep = exp(-h * ikT);
  constexpr int NC = MU_P - MU_U;                 // points about the root (after the first step)
  double cfac[NC];
  bool cprod = !first;
  if (!first) {
    const double m = xs[MU_U];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double off = c == 0 ? 0.0 : (hi - lo) * __builtin_amdgcn_ldexp(1.0, -20 + 8 * ((c - 1) >> 1));
      const double xc = (c & 1) ? m - off : m + off;
      cprod = cprod && xc == xs[MU_U + c];        // not clamped (uniform over the launch)
      cfac[c] = c == 0 ? 1.0 : exp(((c & 1) ? off : -off) * ikT);
    }
  }
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
      const double z0 = (l - xs[0]) * ikT;
      const double zm = first ? 0.0 : (l - xs[MU_U]) * ikT;
      if (first) even_points<MU_P>(v, xs, l, z0, qstep, ikT, w);
      else even_points<MU_U>(v, xs, l, z0, qstep, ikT, w);
      if (!first) {
        if (cprod && fabs(zm) <= 600.0) {
          const double Em = exp(zm);
#pragma unroll
          for (int c = 0; c < NC; ++c) v[MU_U + c] += 2.0 * rcp_nr(1.0 + fmin(Em * cfac[c], 1e300)) * w;
        } else {
#pragma unroll
          for (int c = 0; c < NC; ++c)
            v[MU_U + c] += 2.0 * rcp_nr(1.0 + fmin(exp((l - xs[MU_U + c]) * ikT), 1e300)) * w;
        }
      }
    }
  }
  store_partials<MU_P, 0>(v, p_out);
}

// mu (the midpoint of the final bracket, or the fixed value), and the
// per-block sums at mu: electron count, band energy, entropy S/k_B (into the
// third partial region).
__global__ void __launch_bounds__(MU_NT) k_mu_final(MuArgs g, int n_iter, double mu_fixed, int fixed) {
  __shared__ double s_mu;
  if (fixed) {
    if (threadIdx.x == 0) s_mu = mu_fixed;
    __syncthreads();
  } else {
    const double* s_in = g.state + MU_STATE0 + 16 * (n_iter & 1);
    const double* p_in = g.partial + (size_t)(n_iter & 1) * MU_NB * MU_PS;
    __shared__ double Np[MU_P];
    const bool done = s_in[MS_DONE] != 0.0;
    if (!done) reduce_partials<MU_P, 0>(p_in, gridDim.x, Np);
    if (threadIdx.x == 0) {
      double s[16], t[16];
      for (int q = 0; q < 16; ++q) s[q] = t[q] = s_in[q];
      if (!done) mu_update(s, Np, g.n_e, t);
      s_mu = 0.5 * (t[MS_LO] + t[MS_HI]);
    }
    __syncthreads();
  }
  const double mu = s_mu;
  if (blockIdx.x == 0 && threadIdx.x == 0) g.state[MU_FINAL] = mu;
  // other blocks of this launch may still be reading the previous partials:
  // the final sums go to a third region behind the two buffers
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
  store_partials<3, 0>(v, g.partial + (size_t)2 * MU_NB * MU_PS);
}

// One block: totals of k_mu_final's partials.
__global__ void __launch_bounds__(MU_NT) k_mu_finish(MuArgs g, int nb) {
  __shared__ double tot[3];
  reduce_partials<3, 0>(g.partial + (size_t)2 * MU_NB * MU_PS, nb, tot);
  if (threadIdx.x == 0) {
    g.eparts[0] = tot[1];      // E_band
    g.eparts[1] = tot[2];      // S / k_B
    g.eparts[3] = tot[0];      // electron count at mu
    if (g.mu_out) *g.mu_out = g.state[MU_FINAL];
  }
}

int mu_blocks(int64_t n_pairs) {
  int64_t b = (n_pairs + MU_NT - 1) / MU_NT;
  if (b > MU_NB) b = MU_NB;
  if (b < 1) b = 1;
  return (int)b;
}

size_t mu_partial_doubles() { return (size_t)3 * MU_NB * MU_PS; }
size_t mu_state_doubles() { return (size_t)MU_STATE0 + 32; }

void launch_mu(const MuArgs& a, double mu_fixed, bool fixed, int n_iter, hipStream_t st) {
  const int nb = mu_blocks(a.n_pairs);
  if (!fixed) {
    hipLaunchKernelGGL(k_mu_bracket, dim3(nb), dim3(MU_NT), 0, st, a);
    for (int it = 0; it < n_iter; ++it) hipLaunchKernelGGL(k_mu_iter, dim3(nb), dim3(MU_NT), 0, st, a, it);
  }
  hipLaunchKernelGGL(k_mu_final, dim3(nb), dim3(MU_NT), 0, st, a, n_iter, mu_fixed, fixed ? 1 : 0);
  hipLaunchKernelGGL(k_mu_finish, dim3(1), dim3(MU_NT), 0, st, a, nb);
}

}  // namespace tbk
