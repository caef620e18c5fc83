// Block Lanczos recursion on every cutoff sphere (Sec. 3, Eqs. 4 and 6-9 in
// block form, seed = the target atom's four orbitals).
//
// One persistent workgroup solves one sphere at a time and takes the next
// atom from a queue. Per block step k (V_k: 4n x 4, n = sphere size):
//   1. W = H V_k                block-sparse, SK blocks rebuilt from the pair
//                               data (h, s), V_k and W in LDS
//   2. A_k = V_k^T W            workgroup reduction (FP64)
//   3. W -= V_k A_k + V_{k-1} B_{k-1}^T          (three-term recursion)
//   4. C = V_{0..k}^T W         one sweep over the stored basis (HBM)
//   5. W -= V_{0..k} C          second sweep, also Gram W^T W and the
//                               column norms before/after (FP64 reductions);
//                               steps 4-5 repeat once if a norm fell by more
//                               than a factor sqrt(2) (twice-is-enough rule)
//   6. W = V_{k+1} B_k          Cholesky QR twice, B_k upper triangular with
//                               positive diagonal; columns whose residual norm
//                               is below tol = 1e-12 ||H^(i)||_F are dropped
//                               (deflation: zero columns, zero rows of B_k)
//                               through a modified Gram-Schmidt fallback.
// The basis V_0..V_k lives in a per-workgroup HBM buffer (the full
// re-orthogonalisation reads it twice per step: the kernel's HBM roofline);
// A_k, B_k go to the projected-matrix buffer, and the rows of V on the rho
// row atoms J = {i} + hop(i) are kept for the density-matrix assembly.
// VT = double (FP64 mode) or float (FP32 mode: basis, W and H.V in FP32 with
// FP32 accumulation; A_k, Gram, norms, Cholesky and B_k stay FP64).
#include "tb_internal.h"

namespace tbk {

constexpr int LZ_NT = 512;
constexpr int LZ_NW = LZ_NT / 64;

template <typename VT> struct Vec4;
template <> struct Vec4<double> { typedef double4 T; };
template <> struct Vec4<float> { typedef float4 T; };


// Sum m values (m <= 16) over the workgroup; result in out[0..m-1] (LDS).
template <int M>
__device__ __forceinline__ void block_sum(double (&v)[M], double* red, double* out) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int q = 0; q < M; ++q) v[q] = wave_sum(v[q]);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < M; ++q) red[wave * 16 + q] = v[q];
  }
  __syncthreads();
  if (tid < M) {
    double s = 0.0;
    for (int w = 0; w < LZ_NW; ++w) s += red[w * 16 + tid];
    out[tid] = s;
  }
  __syncthreads();
}

// Butterfly reduce-scatter of 16 values over a wave; lanes with (lane & 3) == 0
// end with the full sum of value index 8*b5 + 4*b4 + 2*b3 + b2 (bits of lane).
__device__ __forceinline__ double wave_sum16(double (&a)[16], int lane, int& which) {
  double b8[8], b4[4], b2[2], b1;
  {
    const bool h = lane & 32;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double send = h ? a[q] : a[q + 8];
      const double keep = h ? a[q + 8] : a[q];
      b8[q] = keep + __shfl_xor(send, 32, 64);
    }
  }
  {
    const bool h = lane & 16;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double send = h ? b8[q] : b8[q + 4];
      const double keep = h ? b8[q + 4] : b8[q];
      b4[q] = keep + __shfl_xor(send, 16, 64);
    }
  }
  {
    const bool h = lane & 8;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const double send = h ? b4[q] : b4[q + 2];
      const double keep = h ? b4[q + 2] : b4[q];
      b2[q] = keep + __shfl_xor(send, 8, 64);
    }
  }
  {
    const bool h = lane & 4;
    const double send = h ? b2[0] : b2[1];
    const double keep = h ? b2[1] : b2[0];
    b1 = keep + __shfl_xor(send, 4, 64);
  }
  b1 += __shfl_xor(b1, 2, 64);
  b1 += __shfl_xor(b1, 1, 64);
  which = 8 * ((lane >> 5) & 1) + 4 * ((lane >> 4) & 1) + 2 * ((lane >> 3) & 1) + ((lane >> 2) & 1);
  return b1;
}

template <typename VT>
__device__ __forceinline__ void load4(const VT* p, double (&v)[4]) {
  typedef typename Vec4<VT>::T V4;
  const V4 x = *(const V4*)p;
  v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
}
template <typename VT>
__device__ __forceinline__ void store4(VT* p, const double (&v)[4]) {
  typedef typename Vec4<VT>::T V4;
  V4 x;
  x.x = (VT)v[0]; x.y = (VT)v[1]; x.z = (VT)v[2]; x.w = (VT)v[3];
  *(V4*)p = x;
}

// In-place Cholesky of the active submatrix of a 4x4 SPD Gram G = U^T U;
// returns false if an active pivot is not safely positive.
__device__ __forceinline__ bool chol4(const double* G, const bool* act, double (&U)[16],
                                      double tol2) {
  for (int q = 0; q < 16; ++q) U[q] = 0.0;
  for (int c = 0; c < 4; ++c) {
    if (!act[c]) continue;
    double d = G[c * 4 + c];
    for (int p = 0; p < c; ++p) if (act[p]) d -= U[p * 4 + c] * U[p * 4 + c];
    if (!(d > 1e-8 * G[c * 4 + c]) || !(d > tol2)) return false;
    const double u = sqrt(d);
    U[c * 4 + c] = u;
    for (int e = c + 1; e < 4; ++e) {
      if (!act[e]) continue;
      double s = G[c * 4 + e];
      for (int p = 0; p < c; ++p) if (act[p]) s -= U[p * 4 + c] * U[p * 4 + e];
      U[c * 4 + e] = s / u;
    }
  }
  return true;
}

// Inverse of an upper-triangular 4x4 restricted to active columns (zero elsewhere).
__device__ __forceinline__ void inv_upper4(const double (&U)[16], const bool* act, double (&X)[16]) {
  for (int q = 0; q < 16; ++q) X[q] = 0.0;
  for (int c = 3; c >= 0; --c) {
    if (!act[c]) continue;
    X[c * 4 + c] = 1.0 / U[c * 4 + c];
    for (int e = c + 1; e < 4; ++e) {
      if (!act[e]) continue;
      double s = 0.0;
      for (int p = c + 1; p <= e; ++p) if (act[p]) s += U[c * 4 + p] * X[p * 4 + e];
      X[c * 4 + e] = -s / U[c * 4 + c];
    }
  }
}

template <typename VT>
__global__ void __launch_bounds__(LZ_NT)
k_lanczos(LanczosArgs g) {
  extern __shared__ unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ncap = g.nc_max, Rcap = 4 * ncap;
  // LDS layout
  VT* s_V = (VT*)smem;                                      // [Rcap][4] current V_k
  VT* s_W = s_V + (size_t)Rcap * 4;                         // [Rcap][4]
  double* s_C = (double*)(((uintptr_t)(s_W + (size_t)Rcap * 4) + 15) & ~(uintptr_t)15);
  // s_C: [max(r_max, LZ_NW)][16] projection coefficients / partials
  const int cslots = (g.r_max > 2 * LZ_NW ? g.r_max : 2 * LZ_NW);
  double* s_Cp = s_C + (size_t)cslots * 16;                 // partials [2*LZ_NW][16]
  double* s_red = s_Cp + (size_t)2 * LZ_NW * 16;            // [LZ_NW][16]
  double* s_misc = s_red + LZ_NW * 16;                      // 128 doubles
  int* s_off = (int*)(s_misc + 128);                        // [ncap+1]
  int* s_gid = s_off + ncap + 1;                            // [ncap]
  signed char* s_js = (signed char*)(s_gid + ncap);         // [ncap]
  __shared__ int s_atom;

  double* A = s_misc;          // [16]
  double* Bp = s_misc + 16;    // [16] previous B
  double* G = s_misc + 32;     // [16] Gram / norms
  double* B = s_misc + 48;     // [16] new B
  double* X = s_misc + 64;     // [16] scratch
  int* s_flag = (int*)(s_misc + 96);     // [8]: active columns, ok, ...

  VT* vbase = (VT*)g.vbuf + (size_t)blockIdx.x * g.r_max * Rcap * 4;
  const VT* pairs = (const VT*)g.pair;

  for (;;) {
    if (tid == 0) s_atom = atomicAdd(g.counter, 1);
    __syncthreads();
    const int atom = s_atom;
    if (atom >= g.n_atoms) break;
    const int n = g.clu_n[atom];
    const int R = 4 * n;
    int r_i = g.r_per_atom ? g.r_per_atom[atom] : g.r_default;
    r_i = r_i < 1 ? 1 : (r_i > g.r_max ? g.r_max : r_i);       // device data: clamp to capacity
    const double tol = 1e-12 * g.hnorm[atom];
    const int* off_g = g.loc_off + (int64_t)atom * (ncap + 1);
    const uint16_t* ent = g.loc_ent + (int64_t)atom * g.emax;
    for (int a = tid; a <= n; a += LZ_NT) s_off[a] = off_g[a];
    for (int a = tid; a < n; a += LZ_NT) { s_gid[a] = g.clu_j[(int64_t)atom * ncap + a]; s_js[a] = -1; }
    __syncthreads();
    const int nh = g.hop_n[s_gid[0]];
    if (tid <= nh) { const int la = g.jloc[(int64_t)atom * JMAX + tid]; if (la >= 0) s_js[la] = (signed char)tid; }
    // seed block V_0 = Phi (target orbitals = rows 0..3)
    for (int row = tid; row < R; row += LZ_NT) {
      double v[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) v[c] = (row == c) ? 1.0 : 0.0;
      store4<VT>(s_V + 4 * row, v);
      store4<VT>(vbase + 4 * row, v);
    }
    if (tid < 16) Bp[tid] = 0.0;
    if (tid < 4) s_flag[tid] = 1;
    __syncthreads();
    VT* vjrow = (VT*)g.vj + (size_t)atom * (4 * JMAX) * (4 * g.r_max);
    const int vjld = 4 * g.r_max;
    // J rows of V_0
    for (int row = tid; row < 4 * JMAX; row += LZ_NT) {
#pragma unroll
      for (int c = 0; c < 4; ++c) vjrow[(size_t)row * vjld + c] = (VT)((row == c) ? 1.0 : 0.0);
    }
    int k_end = r_i;
    int ndefl = 0, n2 = 0;
    double* tab = g.tab + (size_t)atom * g.r_max * 32;

    for (int k = 0; k < r_i; ++k) {
      const VT* Vk = vbase + (size_t)k * Rcap * 4;
      // ---- 1. W = H V_k
      for (int item = tid; item < 4 * n; item += LZ_NT) {
        const int a = item >> 2, c = item & 3;
        const VT* va = s_V + 16 * a + c;
        const VT es = (VT)g.eps_s, ep = (VT)g.eps_p, vsss = (VT)g.v_sss, vsps = (VT)g.v_sps,
                 vdif = (VT)(g.v_pps - g.v_ppp), vppp = (VT)g.v_ppp;
        VT w0 = es * va[0], w1 = ep * va[4], w2 = ep * va[8], w3 = ep * va[12];
        const int gid = s_gid[a];
        int e1 = s_off[a + 1];
        if (e1 > g.emax) e1 = (int)g.emax;
        for (int e = s_off[a]; e < e1; ++e) {
          const unsigned int pe = ent[e];
          const int b = pe & NCLUSTER_LIMIT, slot = pe >> LOCAL_BITS;
          typedef typename Vec4<VT>::T V4;
          const V4 hp4 = *(const V4*)(pairs + ((size_t)gid * ZMAX + slot) * 4);
          const VT hx = hp4.x, hy = hp4.y, hz = hp4.z, s = hp4.w;
          const VT* vb = s_V + 16 * b + c;
          const VT vs = vb[0], vx = vb[4], vy = vb[8], vz = vb[12];
          const VT hp = hx * vx + hy * vy + hz * vz;
          w0 += s * (vsss * vs + vsps * hp);
          const VT t = s * (vdif * hp - vsps * vs);
          const VT sp = s * vppp;
          w1 += t * hx + sp * vx;
          w2 += t * hy + sp * vy;
          w3 += t * hz + sp * vz;
        }
        VT* wa = s_W + 16 * a + c;
        wa[0] = w0; wa[4] = w1; wa[8] = w2; wa[12] = w3;
      }
      __syncthreads();
      // ---- 2. A_k = V_k^T W
      {
        double acc[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = 0.0;
        for (int row = tid; row < R; row += LZ_NT) {
          double v[4], w[4];
          load4<VT>(s_V + 4 * row, v);
          load4<VT>(s_W + 4 * row, w);
#pragma unroll
          for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int d = 0; d < 4; ++d) acc[c * 4 + d] += v[c] * w[d];
        }
        block_sum<16>(acc, s_red, X);
        if (tid < 16) {
          const int c = tid >> 2, d = tid & 3;
          const double a = 0.5 * (X[c * 4 + d] + X[d * 4 + c]);
          A[tid] = a;
          tab[(size_t)k * 32 + tid] = a;
        }
        __syncthreads();
      }
      if (k == r_i - 1) break;
      // ---- 3. three-term recursion
      {
        const VT* Vprev = (k > 0) ? vbase + (size_t)(k - 1) * Rcap * 4 : nullptr;
        for (int row = tid; row < R; row += LZ_NT) {
          double v[4], w[4], vp[4] = {0, 0, 0, 0};
          load4<VT>(s_V + 4 * row, v);
          load4<VT>(s_W + 4 * row, w);
          if (Vprev) load4<VT>(Vprev + 4 * row, vp);
#pragma unroll
          for (int d = 0; d < 4; ++d) {
            double t = w[d];
#pragma unroll
            for (int c = 0; c < 4; ++c) t -= v[c] * A[c * 4 + d] + vp[c] * Bp[d * 4 + c];
            w[d] = t;
          }
          store4<VT>(s_W + 4 * row, w);
        }
        __syncthreads();
      }
      // ---- 4/5. full re-orthogonalisation against V_0..V_k (one pass, a
      // second one if a column norm dropped by more than sqrt(2))
      for (int pass = 0; pass < 2; ++pass) {
        const int nb = k + 1;
        const int parts = (nb >= LZ_NW) ? 1 : (2 * LZ_NW) / nb;   // row splits per block
        const int items = nb * parts;
        for (int it = wave; it < items; it += LZ_NW) {
          const int j = it / parts, part = it % parts;
          const VT* Vj = vbase + (size_t)j * Rcap * 4;
          VT pacc[16];
#pragma unroll
          for (int q = 0; q < 16; ++q) pacc[q] = (VT)0;
          for (int row = part * 64 + lane; row < R; row += 64 * parts) {
            typedef typename Vec4<VT>::T V4;
            const V4 v = *(const V4*)(Vj + 4 * row);
            const V4 w = *(const V4*)(s_W + 4 * row);
            const VT vv[4] = {v.x, v.y, v.z, v.w}, ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
              for (int d = 0; d < 4; ++d) pacc[c * 4 + d] += vv[c] * ww[d];
          }
          double acc[16];
#pragma unroll
          for (int q = 0; q < 16; ++q) acc[q] = (double)pacc[q];
          int which;
          const double sum = wave_sum16(acc, lane, which);
          if ((lane & 3) == 0) {
            if (parts == 1) s_C[j * 16 + which] = sum;
            else s_Cp[it * 16 + which] = sum;
          }
        }
        __syncthreads();
        if (parts > 1) {
          for (int q = tid; q < nb * 16; q += LZ_NT) {
            const int j = q >> 4, e = q & 15;
            double s = 0.0;
            for (int p = 0; p < parts; ++p) s += s_Cp[(j * parts + p) * 16 + e];
            s_C[q] = s;
          }
          __syncthreads();
        }
        // update sweep with Gram (10) and norms-before (4)
        double acc[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = 0.0;
        for (int row = tid; row < R; row += LZ_NT) {
          typedef typename Vec4<VT>::T V4;
          const V4 w4 = *(const V4*)(s_W + 4 * row);
          VT w[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
          for (int d = 0; d < 4; ++d) acc[12 + d] += (double)w[d] * (double)w[d];
          int j = 0;
          for (; j + 1 < nb; j += 2) {
            const V4 a0 = *(const V4*)(vbase + (size_t)j * Rcap * 4 + 4 * row);
            const V4 a1 = *(const V4*)(vbase + (size_t)(j + 1) * Rcap * 4 + 4 * row);
            const VT v0[4] = {a0.x, a0.y, a0.z, a0.w}, v1[4] = {a1.x, a1.y, a1.z, a1.w};
            const double* C0 = s_C + j * 16;
            const double* C1 = s_C + (j + 1) * 16;
#pragma unroll
            for (int d = 0; d < 4; ++d) {
              VT t = w[d];
#pragma unroll
              for (int c = 0; c < 4; ++c) t -= v0[c] * (VT)C0[c * 4 + d] + v1[c] * (VT)C1[c * 4 + d];
              w[d] = t;
            }
          }
          if (j < nb) {
            const V4 a0 = *(const V4*)(vbase + (size_t)j * Rcap * 4 + 4 * row);
            const VT v0[4] = {a0.x, a0.y, a0.z, a0.w};
            const double* C0 = s_C + j * 16;
#pragma unroll
            for (int d = 0; d < 4; ++d) {
              VT t = w[d];
#pragma unroll
              for (int c = 0; c < 4; ++c) t -= v0[c] * (VT)C0[c * 4 + d];
              w[d] = t;
            }
          }
          V4 wo; wo.x = w[0]; wo.y = w[1]; wo.z = w[2]; wo.w = w[3];
          *(V4*)(s_W + 4 * row) = wo;
          const double w0 = w[0], w1 = w[1], w2 = w[2], w3 = w[3];
          acc[0] += w0 * w0; acc[1] += w0 * w1; acc[2] += w0 * w2; acc[3] += w0 * w3;
          acc[4] += w1 * w1; acc[5] += w1 * w2; acc[6] += w1 * w3;
          acc[7] += w2 * w2; acc[8] += w2 * w3; acc[9] += w3 * w3;
        }
        block_sum<16>(acc, s_red, X);
        if (tid == 0) {
          const int map[16] = {0, 1, 2, 3, 1, 4, 5, 6, 2, 5, 7, 8, 3, 6, 8, 9};
          for (int q = 0; q < 16; ++q) G[q] = X[map[q]];
          int again = 0;
          for (int d = 0; d < 4; ++d)
            if (s_flag[d] && X[12 + d] > tol * tol && G[d * 4 + d] < 0.5 * X[12 + d]) again = 1;
          s_flag[4] = again;
        }
        __syncthreads();
        if (!s_flag[4] || pass == 1) break;
        ++n2;
      }
      // ---- 6. QR of W: Cholesky QR twice, or MGS with deflation
      if (tid == 0) {
        bool act[4];
        for (int c = 0; c < 4; ++c) act[c] = s_flag[c] != 0;
        double U[16], Ui[16];
        const bool ok = chol4(G, act, U, tol * tol);
        s_flag[5] = ok ? 1 : 0;
        if (ok) {
          inv_upper4(U, act, Ui);
          for (int q = 0; q < 16; ++q) { B[q] = U[q]; X[q] = Ui[q]; }
        }
      }
      __syncthreads();
      if (s_flag[5]) {
        // V = W U^-1, Gram of V, second Cholesky
        double acc[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = 0.0;
        for (int row = tid; row < R; row += LZ_NT) {
          double w[4], v[4];
          load4<VT>(s_W + 4 * row, w);
#pragma unroll
          for (int d = 0; d < 4; ++d) {
            double t = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) t += w[c] * X[c * 4 + d];
            v[d] = t;
          }
          store4<VT>(s_W + 4 * row, v);
          acc[0] += v[0] * v[0]; acc[1] += v[0] * v[1]; acc[2] += v[0] * v[2]; acc[3] += v[0] * v[3];
          acc[4] += v[1] * v[1]; acc[5] += v[1] * v[2]; acc[6] += v[1] * v[3];
          acc[7] += v[2] * v[2]; acc[8] += v[2] * v[3]; acc[9] += v[3] * v[3];
        }
        block_sum<16>(acc, s_red, G);
        if (tid == 0) {
          const int map[16] = {0, 1, 2, 3, 1, 4, 5, 6, 2, 5, 7, 8, 3, 6, 8, 9};
          double G2[16];
          for (int q = 0; q < 16; ++q) G2[q] = G[map[q]];
          bool act[4];
          for (int c = 0; c < 4; ++c) act[c] = s_flag[c] != 0;
          double U[16], Ui[16];
          chol4(G2, act, U, 0.0);
          inv_upper4(U, act, Ui);
          double Bn[16];
          for (int r0 = 0; r0 < 4; ++r0)
            for (int c = 0; c < 4; ++c) {
              double s = 0.0;
              for (int p = 0; p < 4; ++p) s += U[r0 * 4 + p] * B[p * 4 + c];
              Bn[r0 * 4 + c] = s;
            }
          for (int q = 0; q < 16; ++q) { B[q] = Bn[q]; X[q] = Ui[q]; }
        }
        __syncthreads();
        for (int row = tid; row < R; row += LZ_NT) {
          double w[4], v[4];
          load4<VT>(s_W + 4 * row, w);
#pragma unroll
          for (int d = 0; d < 4; ++d) {
            double t = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) t += w[c] * X[c * 4 + d];
            v[d] = t;
          }
          store4<VT>(s_W + 4 * row, v);
        }
      } else {
        // modified Gram-Schmidt (twice) within the block, with deflation
        if (tid < 16) B[tid] = 0.0;
        __syncthreads();
        for (int c = 0; c < 4; ++c) {
          for (int pass = 0; pass < 2; ++pass) {
            for (int p = 0; p < c; ++p) {
              if (!s_flag[p]) continue;          // uniform (LDS)
              double acc[1] = {0.0};
              for (int row = tid; row < R; row += LZ_NT)
                acc[0] += (double)s_W[4 * row + p] * (double)s_W[4 * row + c];
              block_sum<1>(acc, s_red, X);
              const double dot = X[0];
              for (int row = tid; row < R; row += LZ_NT)
                s_W[4 * row + c] = (VT)((double)s_W[4 * row + c] - dot * (double)s_W[4 * row + p]);
              if (tid == 0) B[p * 4 + c] += dot;
              __syncthreads();
            }
          }
          double acc[1] = {0.0};
          for (int row = tid; row < R; row += LZ_NT) acc[0] += (double)s_W[4 * row + c] * (double)s_W[4 * row + c];
          block_sum<1>(acc, s_red, X);
          const double nrm = sqrt(X[0]);
          const bool keep = nrm > tol;
          const double sc = keep ? 1.0 / nrm : 0.0;
          for (int row = tid; row < R; row += LZ_NT) s_W[4 * row + c] = (VT)((double)s_W[4 * row + c] * sc);
          if (tid == 0) {
            if (keep) B[c * 4 + c] = nrm;
            else { for (int e = 0; e < 4; ++e) B[c * 4 + e] = 0.0; }
            if (s_flag[c] && !keep) ++ndefl;
            s_flag[c] = keep ? 1 : 0;
          }
          __syncthreads();
        }
      }
      __syncthreads();
      // ---- store V_{k+1}: LDS current block, HBM basis, J rows; B_k
      {
        VT* Vn = vbase + (size_t)(k + 1) * Rcap * 4;
        for (int row = tid; row < R; row += LZ_NT) {
          double v[4];
          load4<VT>(s_W + 4 * row, v);
          store4<VT>(s_V + 4 * row, v);
          store4<VT>(Vn + 4 * row, v);
          const int js = s_js[row >> 2];
          if (js >= 0) {
            VT* dst = vjrow + (size_t)(4 * js + (row & 3)) * vjld + 4 * (k + 1);
#pragma unroll
            for (int c = 0; c < 4; ++c) dst[c] = (VT)v[c];
          }
        }
        if (tid < 16) {
          tab[(size_t)k * 32 + 16 + tid] = B[tid];
          Bp[tid] = B[tid];
        }
        __syncthreads();
      }
      (void)Vk;
      if (!(s_flag[0] | s_flag[1] | s_flag[2] | s_flag[3])) {   // invariant space
        k_end = k + 1;
        if (tid == 0) atomicAdd((unsigned long long*)&g.stats[ST_EARLY_STOP], 1ull);
        break;
      }
    }
    if (tid == 0) {
      g.kused[atom] = k_end;
      if (ndefl) atomicAdd((unsigned long long*)&g.stats[ST_DEFLATED], (unsigned long long)ndefl);
      if (n2) atomicAdd((unsigned long long*)&g.stats[ST_REORTH2], (unsigned long long)n2);
    }
    __syncthreads();
  }
}

size_t lanczos_lds_bytes(int nc_max, int r_max, bool fp32) {
  const size_t vt = fp32 ? 4 : 8;
  const size_t Rcap = 4 * (size_t)nc_max;
  size_t b = 2 * Rcap * 4 * vt + 16;
  const int cslots = r_max > 2 * LZ_NW ? r_max : 2 * LZ_NW;
  b += (size_t)cslots * 16 * 8 + 2 * LZ_NW * 16 * 8 + LZ_NW * 16 * 8 + 128 * 8;
  b += (size_t)(nc_max + 1) * 4 + (size_t)nc_max * 4 + (size_t)nc_max;
  return b + 64;
}

void launch_lanczos(const LanczosArgs& a, bool fp32, int n_wg, size_t lds, hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(k_lanczos<float>, dim3(n_wg), dim3(LZ_NT), lds, st, a);
  else
    hipLaunchKernelGGL(k_lanczos<double>, dim3(n_wg), dim3(LZ_NT), lds, st, a);
}

hipError_t lanczos_set_lds(size_t lds) {
  hipError_t e = hipFuncSetAttribute((const void*)k_lanczos<double>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_lanczos<float>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

int lanczos_threads() { return LZ_NT; }

}  // namespace tbk
