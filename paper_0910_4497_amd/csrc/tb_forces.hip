// Energies and forces (Sec. 2: <F_i> = Tr[rho F_i] with F_i = -dH/dR_i).
//
// For the ordered pair (i -> j), d = R_j - R_i, H_ij = s(|d|) M(h) with the
// Slater-Koster matrix M(h), and the rho block X = rho_ji^T of seed i,
//   g_ij = d Tr[H_ij rho_ji] / d d
//        = h [s' (V_sss X_ss + V_sps h.u + V_ppp tr X_pp + D h.X_pp.h)
//             - (s/r)(V_sps h.u + 2 D h.X_pp.h)]
//          + (s/r) [V_sps u + D (X_pp h + X_pp^T h)],
// D = V_pps - V_ppp, u_a = X_{s,a} - X_{a,s}. The pair adds +g to the energy
// gradient on R_j and -g on R_i, so for atom k
//   F_k = sum_{j in hop(k)} (g_kj - g_jk) + repulsive part,
// gathered per atom by 16 lanes (no atomics, fixed order). Repulsion
// E_rep = sum_i F(x_i), x_i = sum_j phi(r_ij), gives
//   F_k += sum_j (F'(x_k) + F'(x_j)) phi'(r_kj) d_kj / r_kj.
// Virial (pressure of the diamond cell, Sec. 5): with the same pair terms,
//   W_ab = sum over ordered pairs (k, j) of (d_kj)_a [g_kj + F'(x_k) phi'(r) d_kj / r]_b,
// each atom summing its own ordered pairs; per-block sums in a fixed order,
// then over blocks in k_energy (bitwise reproducible).
#include <mutex>

#include "tb_internal.h"

namespace tbk {

constexpr int F_NT = 256;


__device__ __forceinline__ void pair_grad(const Model& M, const double* dvec, const double* rho,
                                          double (&g)[3]) {
  const double r = dvec[3];
  double s, ds;
  hop_scale(M, r, s, ds);
  if (s == 0.0 && ds == 0.0) { g[0] = g[1] = g[2] = 0.0; return; }
  const double h[3] = {dvec[0] / r, dvec[1] / r, dvec[2] / r};
  // X[b][a] = rho[a][b]
  double X[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) X[b][a] = rho[a * 4 + b];
  const double D = M.v_pps - M.v_ppp;
  double u[3], Xh[3], XTh[3];
  double hu = 0.0, trp = 0.0, hXh = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    u[a] = X[0][1 + a] - X[1 + a][0];
    hu += h[a] * u[a];
    trp += X[1 + a][1 + a];
    double t1 = 0.0, t2 = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) { t1 += X[1 + a][1 + b] * h[b]; t2 += h[b] * X[1 + b][1 + a]; }
    Xh[a] = t1; XTh[a] = t2;
    hXh += h[a] * t1;
  }
  const double sr = s / r;
  const double radial = ds * (M.v_sss * X[0][0] + M.v_sps * hu + M.v_ppp * trp + D * hXh)
                        - sr * (M.v_sps * hu + 2.0 * D * hXh);
#pragma unroll
  for (int c = 0; c < 3; ++c) g[c] = h[c] * radial + sr * (M.v_sps * u[c] + D * (Xh[c] + XTh[c]));
}

// Sixteen lanes per atom: lane q adds the pair terms of hops q, q + 16, ...,
// the group sums them in a fixed order (shuffles) and its first lane
// evaluates the embedding polynomial.
constexpr int RX_LPA = 16;

__global__ void __launch_bounds__(F_NT) k_rep_x(ForceArgs g) {
  const int gid = blockIdx.x * F_NT + threadIdx.x;
  const int i = gid / RX_LPA, q = gid % RX_LPA;
  double x = 0.0;
  if (i < g.n_atoms) {
    const int nh = g.hop_n[i];
    for (int t = q; t < nh; t += RX_LPA) {
      double phi, dphi;
      pair_term(g.M, g.hop_d[((size_t)i * g.zmax + t) * 4 + 3], phi, dphi);
      x += phi;
    }
  }
#pragma unroll
  for (int off = 1; off < RX_LPA; off <<= 1) x += __shfl_xor(x, off, 64);
  if (i < g.n_atoms && q == 0) {
    const double* c = g.M.frep;
    const double F = c[0] + x * (c[1] + x * (c[2] + x * (c[3] + x * c[4])));
    const double dF = c[1] + x * (2.0 * c[2] + x * (3.0 * c[3] + x * 4.0 * c[4]));
    g.xrep[2 * i] = dF;
    g.xrep[2 * i + 1] = F;
  }
}

// Sixteen lanes per atom: lane q of the group takes hop pairs q, q + 16,
// ... (a hop list is rarely longer than 16, so a lane's pair terms are one
// chain of dependent loads, not several in a row); the group then sums in a
// fixed order (shuffles), so the result does not depend on timing. 64 atoms
// per block of 1024 threads.
constexpr int FF_LPA = 16;                 // lanes per atom
constexpr int FF_NT = 1024;
constexpr int F_APB = FF_NT / FF_LPA;      // atoms per block

__global__ void __launch_bounds__(FF_NT) k_forces(ForceArgs g) {
  __shared__ double s_w[FF_NT / 64][9];
  const int q4 = threadIdx.x & (FF_LPA - 1);
  const int k = blockIdx.x * F_APB + threadIdx.x / FF_LPA;
  double W[9], F[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < 9; ++q) W[q] = 0.0;
  if (k < g.n_atoms) {
    const int nh = g.hop_n[k];
    const int64_t pk = g.row_ptr[k];
    const double dFk = g.xrep[2 * k];
    for (int t = q4; t < nh; t += FF_LPA) {
      const size_t q = (size_t)k * g.zmax + t;
      const int j = g.hop_j[q];
      const double* dv = g.hop_d + 4 * q;
      double gkj[3], gjk[3];
      pair_grad(g.M, dv, g.rho + (size_t)(pk + 1 + t) * 16, gkj);
      const int rt = g.hop_rev[q];
      if (rt >= 0) {
        const size_t qj = (size_t)j * g.zmax + rt;
        pair_grad(g.M, g.hop_d + 4 * qj, g.rho + (size_t)(g.row_ptr[j] + 1 + rt) * 16, gjk);
      } else {
        gjk[0] = gjk[1] = gjk[2] = 0.0;     // only after a list overflow (flagged)
      }
      double phi, dphi;
      pair_term(g.M, dv[3], phi, dphi);
      const double rep = (dFk + g.xrep[2 * j]) * dphi / dv[3];
      const double rep_k = dFk * dphi / dv[3];      // this atom's embedding term of the pair
#pragma unroll
      for (int c = 0; c < 3; ++c) F[c] += gkj[c] - gjk[c] + rep * dv[c];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) W[a * 3 + b] += dv[a] * (gkj[b] + rep_k * dv[b]);
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int off = 1; off < FF_LPA; off <<= 1) F[c] += __shfl_xor(F[c], off, 64);
  }
  if (k < g.n_atoms && q4 == 0 && g.forces) {
    // backward of E_tot: grad_pos = -g F with the upstream gradient g
    const double sc = g.grad_scale ? -*g.grad_scale : 1.0;
    g.forces[3 * k] = sc * F[0];
    g.forces[3 * k + 1] = sc * F[1];
    g.forces[3 * k + 2] = sc * F[2];
  }
  {
    // the nine sums over the wave by the reduce-scatter of wave_sum16 (its
    // pairwise additions are those of wave_sum, in the same order)
    double a[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) a[q] = q < 9 ? W[q] : 0.0;
    int which;
    const int lane = threadIdx.x & 63;
    const double sum = wave_sum16(a, lane, which);
    if ((lane & 3) == 0 && which < 9) s_w[threadIdx.x >> 6][which] = sum;
  }
  __syncthreads();
  if (threadIdx.x < 9) {
    double t = 0.0;
    for (int w = 0; w < FF_NT / 64; ++w) t += s_w[w][threadIdx.x];
    g.wpart[(size_t)blockIdx.x * 9 + threadIdx.x] = t;
  }
}

// Single block: fixed-order sums of the per-atom repulsive energies and of
// the per-block virials (when k_forces ran), then the energy record.
__global__ void __launch_bounds__(F_NT) k_energy(ForceArgs g, int with_virial) {
  __shared__ double red[F_NT / 64];
  if (with_virial && threadIdx.x < 9) {     // virial: blocks in a fixed order
    const int nb = (g.n_atoms + F_APB - 1) / F_APB;
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += g.wpart[(size_t)b * 9 + threadIdx.x];
    g.virial[threadIdx.x] = t;
  }
  double s = 0.0;
  for (int i = threadIdx.x; i < g.n_atoms; i += F_NT) s += g.xrep[2 * i + 1];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0 && g.e_out) {
    double e = 0.0;
    for (int w = 0; w < F_NT / 64; ++w) e += red[w];
    const double eb = g.eparts[0], ts = -g.kT * g.eparts[1];
    g.eparts[2] = e;
    g.e_out[0] = eb;
    g.e_out[1] = ts;
    g.e_out[2] = e;
    g.e_out[3] = eb + ts + e;
  }
}

void launch_forces(const ForceArgs& a, bool with_forces, hipStream_t st) {
  const int nb = (int)(((int64_t)a.n_atoms * RX_LPA + F_NT - 1) / F_NT);
  hipLaunchKernelGGL(k_rep_x, dim3(nb), dim3(F_NT), 0, st, a);
  if (with_forces)
    hipLaunchKernelGGL(k_forces, dim3((a.n_atoms + F_APB - 1) / F_APB), dim3(FF_NT), 0, st, a);
  hipLaunchKernelGGL(k_energy, dim3(1), dim3(F_NT), 0, st, a, with_forces ? 1 : 0);
}

// ------------------------------------------------ fixed device workspace
// tb_energy_forces_static runs the kernels above with their partial results
// -- the per-atom repulsion staging xrep [N][2] and the per-block virial sums
// wpart [ceil(N/64)][9] -- in this file-scope array instead of the context's
// workspace, for callers that cannot allocate. Every element a call reads is
// written earlier in the same call, so nothing needs clearing; calls that
// overlap on one device share the array and race. Host code never uses the
// array's name as an address: each device's address comes from
// hipGetSymbolAddress, taken once per device at context creation.
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)2 << 20;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

constexpr int SCRATCH_DEVICES = 64;
static void* g_scratch_ptr[SCRATCH_DEVICES];
static std::mutex g_scratch_mu;

hipError_t static_scratch_init(int device) {
  if (device < 0 || device >= SCRATCH_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;       // the caller makes `device` current
  void* ptr = nullptr;
  e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t static_scratch_need(int64_t n_atoms) {
  const int64_t nb = (n_atoms + F_APB - 1) / F_APB;
  return align256((size_t)n_atoms * 2 * sizeof(double)) + align256((size_t)nb * 9 * sizeof(double));
}
size_t static_scratch_bytes() { return STATIC_SCRATCH_BYTES; }

bool static_scratch_args(int device, ForceArgs& a) {
  if (device < 0 || device >= SCRATCH_DEVICES) return false;
  unsigned char* base;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    base = (unsigned char*)g_scratch_ptr[device];
  }
  if (!base) return false;
  a.xrep = (double*)base;
  a.wpart = (double*)(base + align256((size_t)a.n_atoms * 2 * sizeof(double)));
  return true;
}

__global__ void k_copy9(const double* __restrict__ src, double* __restrict__ dst) {
  if (threadIdx.x < 9) dst[threadIdx.x] = src[threadIdx.x];
}

void launch_virial_copy(const double* src, double* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_copy9, dim3(1), dim3(64), 0, st, src, dst);
}

}  // namespace tbk
