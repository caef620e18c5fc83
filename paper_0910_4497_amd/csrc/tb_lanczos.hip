// Block Lanczos recursion on every cutoff sphere (Sec. 3, Eqs. 4 and 6-9 in
// block form, seed = the target atom's four orbitals).
//
// One persistent workgroup solves one sphere at a time and takes the next
// atom from a queue. Per block step k (V_k: 4n x 4, n = sphere size):
//   1. W = H V_k and A_k = V_k^T W: block-sparse H.V with the SK blocks
//      rebuilt from the pair data (h, s), V_k and W in LDS; A_k by a
//      workgroup reduction (FP64).
//   2. W -= V_k A_k + V_{k-1} B_{k-1}^T (three-term recursion), with the Gram
//      matrix W^T W.
//   3. A running estimate of |V_j^T V_{k+1}| for every j <= k (block form of
//      Simon's recurrence, kept in FP32). When it exceeds eta (1e-12 FP64,
//      1e-4 FP32), C = V_{0..k}^T W and W -= V_{0..k} C: two sweeps over the
//      stored basis (HBM), for this block and the next, repeated once if a
//      column norm fell by more than a factor sqrt(2).
//   4. W = V_{k+1} B_k by Cholesky QR (twice when the pivots are poorly
//      separated), B_k upper triangular with positive diagonal; a modified
//      Gram-Schmidt fallback drops columns whose residual norm is below
//      tol = 1e-12 ||H^(i)||_F (deflation: zero columns, zero rows of B_k).
//   5. V_{k+1} to LDS (the next step's V_k), to the basis buffer and to the
//      rows on the rho row atoms J = {i} + hop(i).
// With orbital seeds (LanczosArgs::scalar) the four columns are four scalar
// chains: A_k and B_k diagonal, each chain re-orthogonalised against its
// own vectors, and only a chain's own entries enter the estimate.
// H.V work items: one column of one atom per lane (FP32), or all four
// columns of every fourth coupling per lane with a reduce-scatter over the
// four lanes (FP64, and the WIDE FP32 variant), or (MF, FP32) the 4x4 blocks
// of 16 target atoms per wave on the matrix cores, one coupling slot per
// four MFMAs, or (AL, FP32 and FP64) one target atom per lane with all four
// columns of its W block in registers.
// VT = double (FP64 mode) or float (FP32 mode: basis, W and H.V in FP32 with
// FP32 accumulation; A_k, Gram, norms, Cholesky and B_k stay FP64). The
// estimates, FP32 copies of A_j, B_j and a second LDS buffer for V_{k-1} stay
// in LDS when the launch shape leaves room (LanczosArgs::om_lds, ab_lds,
// vprev_lds), else in global memory.
#include "tb_internal.h"

namespace tbk {

// Value of lane C of each quad (4 consecutive lanes), by a DPP broadcast.
template <int C>
__device__ __forceinline__ float quad_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), C * 0x55, 0xF, 0xF, false));
}


// Lane permutations within each quad of lanes (DPP quad_perm, no LDS round
// trip): lane (l & ~3) + P_j's value for the j-th lane of the quad.
template <int PERM>
__device__ __forceinline__ float quad_perm(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), PERM, 0xF, 0xF, false));
}
template <int PERM>
__device__ __forceinline__ double quad_perm(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), PERM, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), PERM, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
constexpr int QP_XOR1 = 0xB1;    // (1, 0, 3, 2)
constexpr int QP_XOR2 = 0x4E;    // (2, 3, 0, 1)

// a * b + c with one rounding
__device__ __forceinline__ float fmav(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmav(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename VT> struct Vec4;
template <> struct Vec4<double> { typedef double4 T; };
template <> struct Vec4<float> { typedef float4 T; };


// Sum m values (m <= 16) over the workgroup; result in out[0..m-1] (LDS).
// FULL: the first barrier is a full one (global stores become visible to the
// workgroup); otherwise both order LDS only.
// More than four values are summed over the wave by the reduce-scatter of
// wave_sum16 (17 shuffles for up to 16 values instead of 6 per value).
template <int M, int NW, bool FULL = false>
__device__ __forceinline__ void block_sum(double (&v)[M], double* red, double* out) {
  static_assert(M <= 16, "at most 16 values");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if constexpr (M > 4) {
    double a[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) a[q] = q < M ? v[q] : 0.0;
    int which;
    const double sum = wave_sum16(a, lane, which);
    if ((lane & 3) == 0 && which < M) red[wave * 16 + which] = sum;
  } else {
#pragma unroll
    for (int q = 0; q < M; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < M; ++q) red[wave * 16 + q] = v[q];
    }
  }
  if (FULL) __syncthreads(); else lds_barrier();
  if (tid < M) {
    double s = 0.0;
    for (int w = 0; w < NW; ++w) s += red[w * 16 + tid];
    out[tid] = s;
  }
  lds_barrier();
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

// Register Cholesky of the active submatrix of a 4x4 SPD Gram G = U^T U;
// false if an active pivot is not safely positive; ratio = min pivot^2 / G_cc.
__device__ __forceinline__ bool chol4r(const double (&G)[16], const bool (&act)[4], double (&U)[16],
                                       double tol2, double& ratio) {
  bool ok = true;
  ratio = 1.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) U[q] = 0.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (!act[c]) continue;
    double d = G[c * 4 + c];
#pragma unroll
    for (int p = 0; p < c; ++p) d -= U[p * 4 + c] * U[p * 4 + c];
    if (!(d > 1e-8 * G[c * 4 + c]) || !(d > tol2)) { ok = false; d = 1.0; }
    const double rr = d / G[c * 4 + c];
    ratio = rr < ratio ? rr : ratio;
    const double u = sqrt(d);
    U[c * 4 + c] = u;
    const double iu = 1.0 / u;
#pragma unroll
    for (int e = c + 1; e < 4; ++e) {
      if (!act[e]) continue;
      double sm = G[c * 4 + e];
#pragma unroll
      for (int p = 0; p < c; ++p) sm -= U[p * 4 + c] * U[p * 4 + e];
      U[c * 4 + e] = sm * iu;
    }
  }
  return ok;
}

__device__ __forceinline__ void inv_upper4r(const double (&U)[16], const bool (&act)[4], double (&X)[16]) {
#pragma unroll
  for (int q = 0; q < 16; ++q) X[q] = 0.0;
#pragma unroll
  for (int c = 3; c >= 0; --c) {
    if (!act[c]) continue;
    const double iu = 1.0 / U[c * 4 + c];
    X[c * 4 + c] = iu;
#pragma unroll
    for (int e = c + 1; e < 4; ++e) {
      if (!act[e]) continue;
      double sm = 0.0;
#pragma unroll
      for (int p = c + 1; p <= e; ++p) sm += U[c * 4 + p] * X[p * 4 + e];
      X[c * 4 + e] = -sm * iu;
    }
  }
}

// LZ_NT threads per workgroup; MINW waves per SIMD the register allocation
// must allow (4: 128 VGPRs, some spilled; 3: 168, with 256 threads, fewer
// spilled; 2: 256 VGPRs, none spilled in FP32). BF
// (with VT = float): the V_k operand of H.V is rounded to BF16 and the
// products with the FP32 Hamiltonian (unrounded on-site and bond parameters
// and pair data) accumulated in FP32; everything else is the FP32
// recursion. WIDE (FP32,
// not BF): the H.V items of the FP64 kernel (each lane all four columns of
// every fourth coupling, then a reduce-scatter over the four lanes), which
// loads each coupling's entry, pair data and V_k rows once instead of once
// per column: the better choice when spheres have many couplings per atom.
template <typename VT, int LZ_NT, int MINW, bool BF = false, bool WIDE = false, bool MF = false, bool AL = false>
__global__ void __launch_bounds__(LZ_NT, MINW)
k_lanczos(LanczosArgs g) {
  static_assert(!BF || sizeof(VT) == 4, "BF16 operands with the FP32 recursion only");
  static_assert(!(BF && WIDE), "the wide H.V items take unrounded operands");
  static_assert(!MF || (sizeof(VT) == 4 && !BF && !WIDE), "the MFMA H.V items are an FP32 layout");
  static_assert(!AL || (!BF && !WIDE && !MF), "one H.V item layout per instance");
  constexpr int LZ_NW = LZ_NT / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ncap = g.nc_max, Rcap = 4 * ncap;
  // LDS layout. Every region is addressed from smem by a byte offset (rounded
  // up to 16 bytes where vector loads need it), so that the compiler keeps the
  // LDS address space of each pointer and emits LDS loads, not flat ones: a
  // flat load's use waits for every global load in flight as well.
  auto at16 = [&](const void* p) {
    return smem + (((size_t)((const unsigned char*)p - smem) + 15) & ~(size_t)15);
  };
  VT* s_Va = (VT*)smem;                                     // [Rcap][4] current V_k
  VT* s_W = s_Va + (size_t)Rcap * 4;                        // [Rcap][4]
  // s_C: [max(r_max, 2 LZ_NW)][16] projection coefficients of a
  // re-orthogonalisation pass in the recursion's precision (they are only
  // used rounded to it), with the FP64 partial sums of a short basis behind
  // the coefficient blocks
  VT* s_C = (VT*)at16(s_W + (size_t)Rcap * 4);
  const int cslots = (g.r_max > 2 * LZ_NW ? g.r_max : 2 * LZ_NW);
  double* s_red = (double*)at16(s_C + (size_t)cslots * 16);  // [LZ_NW][16]
  double* s_misc = s_red + LZ_NW * 16;                      // 224 doubles
  int* s_off = (int*)(s_misc + 224);                        // [ncap+1]
  int* s_gid = s_off + ncap + 1;                            // [ncap]
  int16_t* s_js = (int16_t*)(s_gid + ncap);                 // [ncap] rho row index of a local atom, or -1
  float* s_om = (float*)at16(s_js + ncap);                  // [3][r_max][16] if om_lds
  float* s_ab = s_om + (g.om_lds ? (size_t)3 * g.r_max * 16 : 0);                 // [r_max][32] if ab_lds
  // second block buffer (vprev_lds): V_k and V_{k+1} alternate, so the
  // three-term update reads V_{k-1} from LDS instead of HBM
  VT* s_Vb = g.vprev_lds ? (VT*)at16(s_ab + (g.ab_lds ? (size_t)g.r_max * 32 : 0))
                         : s_Va;
  __shared__ int s_atom;

  double* A = s_misc;          // [16]
  double* Bp = s_misc + 16;    // [16] previous B
  double* G = s_misc + 32;     // [16] Gram / norms
  double* B = s_misc + 48;     // [16] new B
  double* X = s_misc + 64;     // [16] scratch
  int* s_flag = (int*)(s_misc + 96);     // [8]: active columns, ok, ...
  double* s_Np = s_misc + 128;           // [16 parts][4] column-norm partials

  VT* vbase = (VT*)g.vbuf + (size_t)blockIdx.x * g.r_max * Rcap * 4;
  const VT* pairs = (const VT*)g.pair;

  for (;;) {
    if (tid == 0) s_atom = atomicAdd(g.counter, 1);
    __syncthreads();
    const int atom = g.atom0 + s_atom;
    if (atom >= g.n_atoms) break;
    const int n = g.clu_n[atom];
    const int R = 4 * n;
    int r_i = g.r_per_atom ? g.r_per_atom[atom] : g.r_default;
    r_i = r_i < 1 ? 1 : (r_i > g.r_max ? g.r_max : r_i);       // device data: clamp to capacity
    const double tol = 1e-12 * g.hnorm[atom];
    const int* off_g = g.loc_off + (int64_t)atom * (ncap + 1);
    const uint32_t* ent = g.loc_ent + (int64_t)atom * g.emax;
    const int jmax = g.zmax + 1;
    for (int a = tid; a <= n; a += LZ_NT) s_off[a] = off_g[a];
    for (int a = tid; a < n; a += LZ_NT) { s_gid[a] = g.clu_j[(int64_t)atom * ncap + a]; s_js[a] = -1; }
    __syncthreads();
    const int nh = g.hop_n[s_gid[0]];
    for (int t = tid; t <= nh; t += LZ_NT) {
      const int la = g.jloc[(int64_t)atom * jmax + t];
      if (la >= 0) s_js[la] = (int16_t)t;
    }
    // seed block V_0 = Phi (target orbitals = rows 0..3)
    for (int row = tid; row < R; row += LZ_NT) {
      double v[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) v[c] = (row == c) ? 1.0 : 0.0;
      store4<VT>(s_Va + 4 * row, v);
      store4<VT>(vbase + 4 * row, v);
    }
    if (tid < 16) Bp[tid] = 0.0;
    if (tid < 4) s_flag[tid] = 1;
    if (tid == 0) s_misc[208] = 0.0;             // running bound of ||T||
    __syncthreads();
    VT* vjrow = (VT*)g.vj + (size_t)atom * (4 * jmax) * (4 * g.r_max);
    const int vjld = 4 * g.r_max;
    // J rows of V_0
    for (int row = tid; row < 4 * jmax; row += LZ_NT) {
#pragma unroll
      for (int c = 0; c < 4; ++c) vjrow[(size_t)row * vjld + c] = (VT)((row == c) ? 1.0 : 0.0);
    }
    int k_end = r_i;
    int ndefl = 0, n2 = 0, nreorth = 0;
    int64_t bytes = (int64_t)R * 4 * (int64_t)sizeof(VT);    // V_0
    bool force_next = false;
    double* tab = g.tab + (size_t)atom * g.r_max * 32;
    const int cq = tid & 3;                 // fixed column of this thread in the H.V items

    for (int k = 0; k < r_i; ++k) {
      VT* s_V = (k & 1) ? s_Vb : s_Va;           // V_k
      VT* s_Vo = (k & 1) ? s_Va : s_Vb;          // V_{k-1}, then V_{k+1} (vprev_lds)
      // ---- 1. W = H V_k, fused with the partial sums of A_k = V_k^T W
      {
        double accA[4] = {0.0, 0.0, 0.0, 0.0};     // A[c'][cq], c' = 0..3
        auto op = [](VT x) -> VT {                 // the V_k operand of the H.V products
          if constexpr (BF) return bf16_round(x); else return x;
        };
        const VT es = (VT)g.eps_s, ep = (VT)g.eps_p, vsss = (VT)g.v_sss, vsps = (VT)g.v_sps,
                 vdif = (VT)(g.v_pps - g.v_ppp), vppp = (VT)g.v_ppp;
        typedef typename Vec4<VT>::T V4;
        // FP64: item (a, part) -- the four lanes of atom a take every fourth
        // coupling and compute all four columns, then a reduce-scatter over the
        // four lanes leaves lane `part` with column c = part (fewer dependent
        // load rounds). FP32: item (a, c) -- one column per lane over all the
        // couplings of atom a (fewer registers).
        if constexpr (AL) {
          // one target atom per lane: all four columns of W[a] (4 x 4) in
          // registers over all of atom a's couplings, in groups of four whose
          // pair data load together with the next group's entries; no
          // reduction over lanes for W, and the partial sums of A_k = V_k^T W
          // as 16 values per lane
          double acc16[16];
#pragma unroll
          for (int q = 0; q < 16; ++q) acc16[q] = 0.0;
          for (int a = tid; a < n; a += LZ_NT) {
            VT w[16];                                 // [orbital][column]
            V4 va[4];
#pragma unroll
            for (int o = 0; o < 4; ++o) {
              va[o] = *(const V4*)(s_V + 16 * a + 4 * o);
              const VT eo = o == 0 ? es : ep;
              w[o * 4] = eo * va[o].x; w[o * 4 + 1] = eo * va[o].y; w[o * 4 + 2] = eo * va[o].z;
              w[o * 4 + 3] = eo * va[o].w;
            }
            const int gid = s_gid[a];
            const int e0 = s_off[a];
            int e1 = s_off[a + 1];
            if (e1 > g.emax) e1 = (int)g.emax;
            unsigned int pe[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) pe[u] = (e0 + u < e1) ? ent[e0 + u] : 0u;
            for (int eg = e0; eg < e1; eg += 4) {
              V4 hp4[4];
              unsigned int pg[4];
#pragma unroll
              for (int u = 0; u < 4; ++u)
                if (eg + u < e1) hp4[u] = *(const V4*)(pairs + ((size_t)gid * g.zmax + (pe[u] >> LOCAL_BITS)) * 4);
#pragma unroll
              for (int u = 0; u < 4; ++u) pg[u] = (eg + 4 + u < e1) ? ent[eg + 4 + u] : 0u;
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                if (eg + u >= e1) break;
                const int b = pe[u] & NCLUSTER_LIMIT;
                const VT hx = hp4[u].x, hy = hp4[u].y, hz = hp4[u].z, sv = hp4[u].w;
                const V4 vs4 = *(const V4*)(s_V + 16 * b), vx4 = *(const V4*)(s_V + 16 * b + 4),
                         vy4 = *(const V4*)(s_V + 16 * b + 8), vz4 = *(const V4*)(s_V + 16 * b + 12);
                const VT vs[4] = {vs4.x, vs4.y, vs4.z, vs4.w}, vx[4] = {vx4.x, vx4.y, vx4.z, vx4.w},
                         vy[4] = {vy4.x, vy4.y, vy4.z, vy4.w}, vz[4] = {vz4.x, vz4.y, vz4.z, vz4.w};
                const VT css = sv * vsss, csp = sv * vsps, cdf = sv * vdif, sp = sv * vppp;
#pragma unroll
                for (int cc = 0; cc < 4; ++cc) {
                  const VT hp = fmav(hz, vz[cc], fmav(hy, vy[cc], hx * vx[cc]));
                  w[cc] = fmav(csp, hp, fmav(css, vs[cc], w[cc]));
                  const VT t = fmav(-csp, vs[cc], cdf * hp);
                  w[4 + cc] = fmav(sp, vx[cc], fmav(t, hx, w[4 + cc]));
                  w[8 + cc] = fmav(sp, vy[cc], fmav(t, hy, w[8 + cc]));
                  w[12 + cc] = fmav(sp, vz[cc], fmav(t, hz, w[12 + cc]));
                }
              }
#pragma unroll
              for (int u = 0; u < 4; ++u) pe[u] = pg[u];
            }
#pragma unroll
            for (int o = 0; o < 4; ++o) {
              V4 wo;
              wo.x = w[o * 4]; wo.y = w[o * 4 + 1]; wo.z = w[o * 4 + 2]; wo.w = w[o * 4 + 3];
              *(V4*)(s_W + 16 * a + 4 * o) = wo;
              const VT vr[4] = {va[o].x, va[o].y, va[o].z, va[o].w};
#pragma unroll
              for (int c2 = 0; c2 < 4; ++c2)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc16[c2 * 4 + c] += (double)vr[c2] * (double)w[o * 4 + c];
            }
          }
          int which;
          const double sum = wave_sum16(acc16, lane, which);
          if ((lane & 3) == 0) s_red[wave * 16 + which] = sum;
        } else if constexpr (MF) {
          // MFMA items: v_mfma_f32_4x4x1_16b_f32 holds 16 blocks of 4 lanes;
          // block b (lanes 4b .. 4b+3) is target atom a = a0 + b, and per
          // coupling slot s the four products H_ab[:, k] V_b[k, :] (k = 0..3)
          // of atom a's s-th coupling (a -> b) accumulate into its 4x4 block
          // of W: lane 4b + q provides H_ab[q][k] (row q of the Slater-Koster
          // block, built from the pair data) and V_b[k][q], and ends holding
          // W[a][0..3][q], the same values as the one-column item (a, q). The
          // whole wave runs every MFMA (atoms past n and slots past an atom's
          // last coupling feed zero rows of H).
          for (int base = 64 * wave; base < 4 * n; base += LZ_NT) {
            const int item = base + lane, c = cq;
            const bool valid = item < 4 * n;
            const int a = valid ? item >> 2 : 0;
            const int e0 = s_off[a];
            int e1 = valid ? s_off[a + 1] : e0;
            if (e1 > g.emax) e1 = (int)g.emax;
            const int ncp = e1 > e0 ? e1 - e0 : 0;
            int smax = ncp;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) smax = max(smax, __shfl_xor(smax, off, 64));
            smax = __builtin_amdgcn_readfirstlane(smax);          // equal on every lane: a scalar trip count
            const int gid = s_gid[a];
            const VT* va = s_V + 16 * a + c;
            typedef float f4 __attribute__((ext_vector_type(4)));
            f4 acc;
            acc[0] = valid ? es * va[0] : 0.0f;
            acc[1] = valid ? ep * va[4] : 0.0f;
            acc[2] = valid ? ep * va[8] : 0.0f;
            acc[3] = valid ? ep * va[12] : 0.0f;
            unsigned int pn = ncp > 0 ? ent[e0] : 0u;
            for (int sl = 0; sl < smax; ++sl) {
              const bool has = sl < ncp;
              const unsigned int pe = pn;
              pn = (sl + 1 < ncp) ? ent[e0 + sl + 1] : 0u;     // the next entry loads with this pair data
              const int slot = pe >> LOCAL_BITS, b = pe & NCLUSTER_LIMIT;
              const V4 hp4 = *(const V4*)(pairs + ((size_t)gid * g.zmax + slot) * 4);
              const VT hx = hp4.x, hy = hp4.y, hz = hp4.z, sv = has ? hp4.w : (VT)0;
              // row c of H_ab: s row (vsss, vsps h) or p_u row (-vsps h_u, vdif h_u h + vppp e_u)
              const VT hu = c == 1 ? hx : (c == 2 ? hy : hz);
              VT h0, h1, h2, h3;
              if (c == 0) {
                h0 = sv * vsss; h1 = sv * vsps * hx; h2 = sv * vsps * hy; h3 = sv * vsps * hz;
              } else {
                const VT t = sv * vdif * hu;
                h0 = -sv * vsps * hu;
                h1 = t * hx + (c == 1 ? sv * vppp : (VT)0);
                h2 = t * hy + (c == 2 ? sv * vppp : (VT)0);
                h3 = t * hz + (c == 3 ? sv * vppp : (VT)0);
              }
              const VT* vb = s_V + 16 * b + c;
              const VT b0 = vb[0], b1 = vb[4], b2 = vb[8], b3 = vb[12];
              acc = __builtin_amdgcn_mfma_f32_4x4x1f32(h0, b0, acc, 0, 0, 0);
              acc = __builtin_amdgcn_mfma_f32_4x4x1f32(h1, b1, acc, 0, 0, 0);
              acc = __builtin_amdgcn_mfma_f32_4x4x1f32(h2, b2, acc, 0, 0, 0);
              acc = __builtin_amdgcn_mfma_f32_4x4x1f32(h3, b3, acc, 0, 0, 0);
            }
            if (valid) {
              const VT wb[4] = {acc[0], acc[1], acc[2], acc[3]};
              VT* wa = s_W + 16 * a + c;
              wa[0] = wb[0]; wa[4] = wb[1]; wa[8] = wb[2]; wa[12] = wb[3];
#pragma unroll
              for (int beta = 0; beta < 4; ++beta) {
                const V4 vr = *(const V4*)(s_V + 4 * (4 * a + beta));
                accA[0] += (double)vr.x * (double)wb[beta];
                accA[1] += (double)vr.y * (double)wb[beta];
                accA[2] += (double)vr.z * (double)wb[beta];
                accA[3] += (double)vr.w * (double)wb[beta];
              }
            }
          }
        } else {
        // four-column items: entries e0 + 4u (u < 4) of this lane's first
        // group of couplings in an item, loaded during the previous item
        constexpr bool WIDE_ITEMS = sizeof(VT) == 8 || WIDE;
        auto first_group = [&](int it, unsigned int (&pq)[4]) {
          const int an = it < 4 * n ? it >> 2 : 0;
          const int f0 = s_off[an] + cq;
          int f1 = it < 4 * n ? s_off[an + 1] : 0;
          if (f1 > g.emax) f1 = (int)g.emax;
#pragma unroll
          for (int u = 0; u < 4; ++u) pq[u] = (f0 + 4 * u < f1) ? ent[f0 + 4 * u] : 0u;
        };
        unsigned int pfx[4] = {0u, 0u, 0u, 0u};
        if constexpr (WIDE_ITEMS) first_group(tid, pfx);
        for (int item = tid; item < 4 * n; item += LZ_NT) {
          VT w0, w1, w2, w3;
          const int a = item >> 2, c = cq;
          if constexpr (WIDE_ITEMS) {

          VT w[16];                                   // [orbital][column]
          if (c == 0) {
#pragma unroll
            for (int o = 0; o < 4; ++o) {
              const V4 va = *(const V4*)(s_V + 16 * a + 4 * o);
              const VT eo = o == 0 ? es : ep;
              w[o * 4] = eo * va.x; w[o * 4 + 1] = eo * va.y; w[o * 4 + 2] = eo * va.z; w[o * 4 + 3] = eo * va.w;
            }
          } else {
#pragma unroll
            for (int q = 0; q < 16; ++q) w[q] = (VT)0;
          }
          const int gid = s_gid[a];
          int e1 = s_off[a + 1];
          if (e1 > g.emax) e1 = (int)g.emax;
          unsigned int pe[4] = {pfx[0], pfx[1], pfx[2], pfx[3]};
          first_group(item + LZ_NT, pfx);           // the next item's, in flight during this one
          // groups of four of this lane's couplings (every fourth of atom a):
          // their pair data load together, with the entries of the next group
          for (int eg = s_off[a] + c; eg < e1; eg += 16) {
            V4 hp4[4];
            unsigned int pg[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (eg + 4 * u < e1) hp4[u] = *(const V4*)(pairs + ((size_t)gid * g.zmax + (pe[u] >> LOCAL_BITS)) * 4);
#pragma unroll
            for (int u = 0; u < 4; ++u) pg[u] = (eg + 16 + 4 * u < e1) ? ent[eg + 16 + 4 * u] : 0u;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              if (eg + 4 * u >= e1) break;
              const int b = pe[u] & NCLUSTER_LIMIT;
              const VT hx = hp4[u].x, hy = hp4[u].y, hz = hp4[u].z, sv = hp4[u].w;
              const V4 vs4 = *(const V4*)(s_V + 16 * b), vx4 = *(const V4*)(s_V + 16 * b + 4),
                       vy4 = *(const V4*)(s_V + 16 * b + 8), vz4 = *(const V4*)(s_V + 16 * b + 12);
              const VT vs[4] = {vs4.x, vs4.y, vs4.z, vs4.w}, vx[4] = {vx4.x, vx4.y, vx4.z, vx4.w},
                       vy[4] = {vy4.x, vy4.y, vy4.z, vy4.w}, vz[4] = {vz4.x, vz4.y, vz4.z, vz4.w};
              // the radial factor enters the four bond integrals once per
              // coupling, so each column costs 13 multiply-adds
              const VT css = sv * vsss, csp = sv * vsps, cdf = sv * vdif, sp = sv * vppp;
#pragma unroll
              for (int cc = 0; cc < 4; ++cc) {
                const VT hp = fmav(hz, vz[cc], fmav(hy, vy[cc], hx * vx[cc]));
                w[cc] = fmav(csp, hp, fmav(css, vs[cc], w[cc]));
                const VT t = fmav(-csp, vs[cc], cdf * hp);
                w[4 + cc] = fmav(sp, vx[cc], fmav(t, hx, w[4 + cc]));
                w[8 + cc] = fmav(sp, vy[cc], fmav(t, hy, w[8 + cc]));
                w[12 + cc] = fmav(sp, vz[cc], fmav(t, hz, w[12 + cc]));
              }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) pe[u] = pg[u];
          }
          {
            const bool hi = c & 2, lo = c & 1;
            VT h[8];
#pragma unroll
            for (int o = 0; o < 4; ++o)
#pragma unroll
              for (int cc = 0; cc < 2; ++cc) {
                const VT keep = hi ? w[o * 4 + 2 + cc] : w[o * 4 + cc];
                const VT send = hi ? w[o * 4 + cc] : w[o * 4 + 2 + cc];
                h[o * 2 + cc] = keep + quad_perm<QP_XOR2>(send);
              }
            VT r[4];
#pragma unroll
            for (int o = 0; o < 4; ++o) {
              const VT keep = lo ? h[o * 2 + 1] : h[o * 2];
              const VT send = lo ? h[o * 2] : h[o * 2 + 1];
              r[o] = keep + quad_perm<QP_XOR1>(send);
            }
            w0 = r[0]; w1 = r[1]; w2 = r[2]; w3 = r[3];
          }
          } else {

          const VT* va = s_V + 16 * a + c;
          w0 = es * op(va[0]); w1 = ep * op(va[4]); w2 = ep * op(va[8]); w3 = ep * op(va[12]);
          const int gid = s_gid[a];
          int e1 = s_off[a + 1];
          if (e1 > g.emax) e1 = (int)g.emax;
          // the entries of the next group of four couplings are loaded with
          // the pair data of the current one (one dependent round trip per
          // group instead of two)
          unsigned int pe[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) pe[u] = (s_off[a] + u < e1) ? ent[s_off[a] + u] : 0u;
          for (int e0 = s_off[a]; e0 < e1; e0 += 4) {
            V4 hp4[4];
            unsigned int pn[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int slot = pe[u] >> LOCAL_BITS;
              hp4[u] = *(const V4*)(pairs + ((size_t)gid * g.zmax + slot) * 4);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) pn[u] = (e0 + 4 + u < e1) ? ent[e0 + 4 + u] : 0u;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              if (e0 + u >= e1) break;
              const int b = pe[u] & NCLUSTER_LIMIT;
              const VT hx = hp4[u].x, hy = hp4[u].y, hz = hp4[u].z, sv = hp4[u].w;
              const VT* vb = s_V + 16 * b + c;
              const VT vs = op(vb[0]), vx = op(vb[4]), vy = op(vb[8]), vz = op(vb[12]);
              const VT hp = hx * vx + hy * vy + hz * vz;
              w0 += sv * (vsss * vs + vsps * hp);
              const VT t = sv * (vdif * hp - vsps * vs);
              const VT sp = sv * vppp;
              w1 += t * hx + sp * vx;
              w2 += t * hy + sp * vy;
              w3 += t * hz + sp * vz;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) pe[u] = pn[u];
          }
          }
          VT* wa = s_W + 16 * a + c;
          wa[0] = w0; wa[4] = w1; wa[8] = w2; wa[12] = w3;
          const VT wb[4] = {w0, w1, w2, w3};
#pragma unroll
          for (int beta = 0; beta < 4; ++beta) {
            const V4 vr = *(const V4*)(s_V + 4 * (4 * a + beta));
            accA[0] += (double)vr.x * (double)wb[beta];
            accA[1] += (double)vr.y * (double)wb[beta];
            accA[2] += (double)vr.z * (double)wb[beta];
            accA[3] += (double)vr.w * (double)wb[beta];
          }
        }
        }
        // reduce over lanes with equal (lane & 3), then over waves: a
        // reduce-scatter on lane bits 2 and 3 (each lane keeps half of its
        // values and adds its partner's copy of that half), then bits 4 and 5;
        // the pairwise additions are those of a butterfly over offsets 4, 8,
        // 16, 32 in that order. Lane l < 16 ends with value (l >> 2) of
        // column l & 3.
        if constexpr (!AL) {
          const bool h2 = lane & 4, h3 = lane & 8;
          const double k0 = h2 ? accA[1] : accA[0], k1 = h2 ? accA[3] : accA[2];
          const double s0 = h2 ? accA[0] : accA[1], s1 = h2 ? accA[2] : accA[3];
          const double b0 = k0 + __shfl_xor(s0, 4, 64), b1 = k1 + __shfl_xor(s1, 4, 64);
          double t = (h3 ? b1 : b0) + __shfl_xor(h3 ? b0 : b1, 8, 64);
          t += __shfl_xor(t, 16, 64);
          t += __shfl_xor(t, 32, 64);
          if (lane < 16) s_red[wave * 16 + lane] = t;
        }
        lds_barrier();
        if (tid < 16) {
          double sum = 0.0;
          for (int w = 0; w < LZ_NW; ++w) sum += s_red[w * 16 + tid];
          X[tid] = sum;
        }
        lds_barrier();
        if (tid < 16) {
          const int c = tid >> 2, d = tid & 3;
          // orbital seeds: independent scalar chains, A_k diagonal
          const double av = (g.scalar && c != d) ? 0.0 : 0.5 * (X[c * 4 + d] + X[d * 4 + c]);
          A[tid] = av;
          tab[(size_t)k * 32 + tid] = av;
          if (g.ab_lds) s_ab[k * 32 + tid] = (float)av;
        }
        lds_barrier();
      }
      if (k == r_i - 1) break;
      // ---- 2. three-term recursion: W -= V_k A_k + V_{k-1} B_{k-1}^T, with
      // the Gram matrix W^T W of the result
      {
        const VT* Vprev = (k == 0) ? nullptr : (g.vprev_lds ? s_Vo : vbase + (size_t)(k - 1) * Rcap * 4);
        double acc[10];
#pragma unroll
        for (int q = 0; q < 10; ++q) acc[q] = 0.0;
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
          load4<VT>(s_W + 4 * row, w);           // the stored (rounded) values
          acc[0] += w[0] * w[0]; acc[1] += w[0] * w[1]; acc[2] += w[0] * w[2]; acc[3] += w[0] * w[3];
          acc[4] += w[1] * w[1]; acc[5] += w[1] * w[2]; acc[6] += w[1] * w[3];
          acc[7] += w[2] * w[2]; acc[8] += w[2] * w[3]; acc[9] += w[3] * w[3];
        }
        // the one full barrier of the step: the global stores of the previous
        // step (V_k, rho rows, A, B, Omega) are visible to the workgroup after it
        block_sum<10, LZ_NW, true>(acc, s_red, G);
        // V_{k+1} written; V_{k-1} read unless it is in LDS
        bytes += (int64_t)R * 4 * (int64_t)sizeof(VT) * (k > 0 && !g.vprev_lds ? 2 : 1);
      }
      // ---- 3a. orthogonality estimate. With Omega_{j,k} = V_j^T V_k, the
      // recursion H V_j = V_{j+1} B_j + V_j A_j + V_{j-1} B_{j-1}^T and the
      // symmetry of H give, for j < k,
      //   Omega_{j,k+1} B_k = B_j^T Omega_{j+1,k} + A_j Omega_{j,k} + B_{j-1} Omega_{j-1,k}
      //                       - Omega_{j,k} A_k - Omega_{j,k-1} B_{k-1}^T  (+ rounding),
      // and Omega_{k,k+1} is of order eps ||H|| / B_k (block form of Simon's
      // recurrence). Rounding is modelled by eps ||T|| added with the sign of
      // each entry; ||T|| is bounded by the running block-Gershgorin row sum.
      // B_k comes from the Cholesky factor of the Gram matrix just formed.
      bool reorth;
      {
        // thread 0: Cholesky factor of the Gram matrix, B_k^-1, ||T|| bound
        double* Xe = s_misc + 192;               // [16] B_k^-1 estimate
        if (tid == 0) {
          double Gf[16], Ur[16], Xr[16], ratio;
          const int map[16] = {0, 1, 2, 3, 1, 4, 5, 6, 2, 5, 7, 8, 3, 6, 8, 9};
          bool actk[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) actk[c] = s_flag[c] != 0;
#pragma unroll
          for (int q = 0; q < 16; ++q) Gf[q] = (g.scalar && q % 5 != 0) ? 0.0 : G[map[q]];
          const bool ok = chol4r(Gf, actk, Ur, tol * tol, ratio);
          inv_upper4r(Ur, actk, Xr);
          double tn = s_misc[208];
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            double rs = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) rs += fabs(A[a * 4 + c]) + fabs(Ur[c * 4 + a]) + fabs(Bp[a * 4 + c]);
            tn = rs > tn ? rs : tn;
          }
#pragma unroll
          for (int q = 0; q < 16; ++q) Xe[q] = Xr[q];
          s_misc[208] = tn;
          s_flag[6] = ok ? 1 : 0;
          if (!g.scalar) {
            // the QR of step 4 factors this same Gram matrix unless a
            // re-orthogonalisation pass changes W first: its factor, inverse
            // and path, ready for that case
#pragma unroll
            for (int q = 0; q < 16; ++q) { X[q] = Xr[q]; B[q] = Ur[q]; }
            s_flag[5] = !ok ? 2 : (ratio > 1e-4 ? 0 : 1);
          }
        }
        lds_barrier();
        const double rnd = 2.0 * g.eps_unit * s_misc[208];
        // one entry (j, a, b) of Omega_{j,k+1} per thread, in FP32 (an
        // estimate); the four lanes holding row (j, a) exchange M by shuffles.
        // The ring of three Omega blocks is in LDS or in global memory; the
        // loop is instantiated for each with pointers of that address space,
        // so that its loads are LDS or global loads (counted in order) rather
        // than flat ones, whose every use waits for all loads in flight.
        const float rndf = (float)rnd;
        double lmax = 0.0;
        const size_t ring = (size_t)g.r_max * 16;
        // LZ_NT is a multiple of 16, so a thread keeps its row a and column b
        // over the loop: its column of A_k, row of B_{k-1} and column of
        // B_k^-1 are read once
        static_assert(LZ_NT % 16 == 0, "entries (j, a, b) keep a and b per thread");
        const int at = (tid >> 2) & 3, bt = tid & 3;
        float Acol[4], Bprow[4], Xcol[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          Acol[c] = (float)A[c * 4 + bt]; Bprow[c] = (float)Bp[bt * 4 + c]; Xcol[c] = (float)Xe[c * 4 + bt];
        }
        auto estimate = [&](auto om, auto tabp) {
          const auto Ok = om + (size_t)(k % 3) * ring;           // Omega_{j,k}, j < k
          const auto Okm = om + (size_t)((k + 2) % 3) * ring;    // Omega_{j,k-1}, j < k-1
          const auto Okp = om + (size_t)((k + 1) % 3) * ring;    // Omega_{j,k+1}, j <= k
          for (int t = tid; t < 16 * (k + 1); t += LZ_NT) {
            const int j = t >> 4, a = at, b = bt;
            // The 16 lanes of block j each load one element (a, b) of every
            // matrix the entry needs, at an in-range block index (the
            // neighbours clamped to [0, k - 1]; k = 0 has no entries j < k),
            // and take the rows and columns they need from the other lanes:
            // within a quad (row a) by DPP broadcasts, across the 16 lanes
            // (column b) by shuffles. The edge cases j = 0, j + 1 = k and
            // j = k - 1 are applied by selects.
            const int jc = j < k ? j : (k > 0 ? k - 1 : 0);
            const int jm = jc > 0 ? jc - 1 : 0, jp = jc + 1 < k ? jc + 1 : jc;
            const int own = a * 4 + b;
            const float w_jk = Ok[jc * 16 + own];      // Omega_{j,k}[a][b]
            const float w_jp = Ok[jp * 16 + own];      // Omega_{j+1,k}[a][b]
            const float w_jm = Ok[jm * 16 + own];      // Omega_{j-1,k}[a][b]
            const float w_l = Okm[jc * 16 + own];      // Omega_{j,k-1}[a][b]
            float ea, eb, ebm;                         // A_j[a][b], B_j[b][a], B_{j-1}[a][b]
            if (g.ab_lds) {
              ea = s_ab[jc * 32 + own]; eb = s_ab[jc * 32 + 16 + b * 4 + a]; ebm = s_ab[jm * 32 + 16 + own];
            } else {
              ea = (float)tabp[jc * 32 + own]; eb = (float)tabp[jc * 32 + 16 + b * 4 + a];
              ebm = (float)tabp[jm * 32 + 16 + own];
            }
            const float aj[4] = {quad_bcast<0>(ea), quad_bcast<1>(ea), quad_bcast<2>(ea), quad_bcast<3>(ea)};
            const float bj[4] = {quad_bcast<0>(eb), quad_bcast<1>(eb), quad_bcast<2>(eb), quad_bcast<3>(eb)};
            const float bjm[4] = {quad_bcast<0>(ebm), quad_bcast<1>(ebm), quad_bcast<2>(ebm), quad_bcast<3>(ebm)};
            const float orow[4] = {quad_bcast<0>(w_jk), quad_bcast<1>(w_jk), quad_bcast<2>(w_jk), quad_bcast<3>(w_jk)};
            const float olast[4] = {quad_bcast<0>(w_l), quad_bcast<1>(w_l), quad_bcast<2>(w_l), quad_bcast<3>(w_l)};
            float ocol[4], onext[4], oprev[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const int src = (lane & ~15) | (c * 4 + b);
              ocol[c] = __shfl(w_jk, src, 64);
              onext[c] = __shfl(w_jp, src, 64);
              oprev[c] = __shfl(w_jm, src, 64);
            }
            float m = rndf;
            if (j < k) {
              float acc = 0.0f;
#pragma unroll
              for (int c = 0; c < 4; ++c) {
                const float ojp = (j + 1 == k) ? (c == b ? 1.0f : 0.0f) : onext[c];
                const float ol = (j == k - 1) ? (a == c ? 1.0f : 0.0f) : olast[c];
                acc += aj[c] * ocol[c] - orow[c] * Acol[c] + bj[c] * ojp - ol * Bprow[c];
                acc += (j > 0) ? bjm[c] * oprev[c] : 0.0f;
              }
              m = acc + copysignf(rndf, acc);
            }
            const float o = quad_bcast<0>(m) * Xcol[0] + quad_bcast<1>(m) * Xcol[1] +
                            quad_bcast<2>(m) * Xcol[2] + quad_bcast<3>(m) * Xcol[3];
            Okp[j * 16 + a * 4 + b] = o;
            // orbital seeds: only a chain's own entries estimate a loss of
            // orthogonality (different chains are not orthogonal)
            if (!g.scalar || a == b) lmax = fmax(lmax, (double)fabsf(o));
          }
        };
        typedef __attribute__((address_space(1))) float g_float;
        typedef __attribute__((address_space(3))) float l_float;
        typedef __attribute__((address_space(1))) const double g_cdouble;
        const auto tab_g = (g_cdouble*)tab;
        if (g.om_lds) estimate((l_float*)s_om, tab_g);
        else estimate((g_float*)((float*)g.omega + (size_t)blockIdx.x * 3 * ring), tab_g);
        lmax = wave_max(lmax);
        if (lane == 0) s_red[wave] = lmax;
        lds_barrier();
        double gmax = 0.0;
        for (int w2 = 0; w2 < LZ_NW; ++w2) gmax = fmax(gmax, s_red[w2]);
        const bool trig = !(gmax <= g.eta) || s_flag[6] == 0;
        reorth = trig || force_next;
        force_next = trig && !force_next;        // a triggered pass also covers the next block
        if (reorth) {
          // the pass restores orthogonality to rounding level (each thread
          // overwrites the entries it stored: the step's barriers order LDS
          // only, and the buffer may be in global memory)
          float* Okp = (g.om_lds ? s_om : (float*)g.omega + (size_t)blockIdx.x * 3 * ring) + (size_t)((k + 1) % 3) * ring;
          for (int t = tid; t < 16 * (k + 1); t += LZ_NT) Okp[t] = (float)g.eps_unit;
          ++nreorth;
        }
        lds_barrier();
      }
      // ---- 3b. when the estimate exceeds eta: full re-orthogonalisation
      // against V_0..V_k: projection sweep (items with block k also give the
      // column norms before the pass), then the update sweep with the Gram
      // matrix of the result; a second pass when a column norm fell by more
      // than sqrt(2).
      for (int pass = 0; reorth && pass < 2; ++pass) {
        const int nb = k + 1;
        bytes += 2 * (int64_t)nb * R * 4 * (int64_t)sizeof(VT);
        // short bases are split over the waves by rows; the partial sums go
        // to the free slots of s_C behind the nb coefficient blocks
        int parts = (nb >= 2 * LZ_NW) ? 1 : (2 * LZ_NW + nb - 1) / nb;
        const int pmax = (int)(((size_t)(cslots - nb) * sizeof(VT) / sizeof(double)) / nb);
        parts = parts <= pmax ? parts : (pmax > 1 ? pmax : 1);
        const int items = nb * parts;
        double* s_Cp = (double*)(s_C + nb * 16);
        for (int it = wave; it < items; it += LZ_NW) {
          const int j = it / parts, part = it % parts;
          const VT* Vj = vbase + (size_t)j * Rcap * 4;
          VT pacc[16];
#pragma unroll
          for (int q = 0; q < 16; ++q) pacc[q] = (VT)0;
          double nacc[4] = {0.0, 0.0, 0.0, 0.0};
          const bool want_norm = (j == k);
          typedef typename Vec4<VT>::T V4;
          const int S = 64 * parts;
          int row = part * 64 + lane;
          constexpr int UP = sizeof(VT) == 8 ? 2 : 4;
          for (; row + (UP - 1) * S < R; row += UP * S) {
            V4 v[UP], w[UP];
#pragma unroll
            for (int u = 0; u < UP; ++u) v[u] = *(const V4*)(Vj + 4 * (row + u * S));
#pragma unroll
            for (int u = 0; u < UP; ++u) w[u] = *(const V4*)(s_W + 4 * (row + u * S));
#pragma unroll
            for (int u = 0; u < UP; ++u) {
              const VT vv[4] = {v[u].x, v[u].y, v[u].z, v[u].w}, ww[4] = {w[u].x, w[u].y, w[u].z, w[u].w};
#pragma unroll
              for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int d = 0; d < 4; ++d) pacc[c * 4 + d] += vv[c] * ww[d];
              if (want_norm) {
#pragma unroll
                for (int d = 0; d < 4; ++d) nacc[d] += (double)ww[d] * (double)ww[d];
              }
            }
          }
          for (; row < R; row += S) {
            const V4 v = *(const V4*)(Vj + 4 * row);
            const V4 w = *(const V4*)(s_W + 4 * row);
            const VT vv[4] = {v.x, v.y, v.z, v.w}, ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
              for (int d = 0; d < 4; ++d) pacc[c * 4 + d] += vv[c] * ww[d];
            if (want_norm) {
#pragma unroll
              for (int d = 0; d < 4; ++d) nacc[d] += (double)ww[d] * (double)ww[d];
            }
          }
          double acc[16];
#pragma unroll
          for (int q = 0; q < 16; ++q) acc[q] = (double)pacc[q];
          int which;
          const double sum = wave_sum16(acc, lane, which);
          if ((lane & 3) == 0) {
            // orbital seeds: a chain is orthogonalised against its own vectors only
            const double cv = (g.scalar && (which >> 2) != (which & 3)) ? 0.0 : sum;
            if (parts == 1) s_C[j * 16 + which] = (VT)cv;
            else s_Cp[it * 16 + which] = cv;
          }
          if (want_norm) {
#pragma unroll
            for (int d = 0; d < 4; ++d) nacc[d] = wave_sum(nacc[d]);
            if (lane < 4) s_Np[part * 4 + lane] = nacc[lane];
          }
        }
        lds_barrier();
        if (parts > 1) {
          for (int q = tid; q < nb * 16; q += LZ_NT) {
            const int j = q >> 4, e = q & 15;
            double sum = 0.0;
            for (int p = 0; p < parts; ++p) sum += s_Cp[(j * parts + p) * 16 + e];
            s_C[q] = (VT)sum;
          }
        }
        if (tid < 4) {
          double sum = 0.0;
          for (int p = 0; p < parts; ++p) sum += s_Np[p * 4 + tid];
          X[12 + tid] = sum;                        // norms before this pass
        }
        lds_barrier();
        // update sweep with the Gram matrix (10 values) of the result
        double acc[10];
#pragma unroll
        for (int q = 0; q < 10; ++q) acc[q] = 0.0;
        for (int row = tid; row < R; row += LZ_NT) {
          typedef typename Vec4<VT>::T V4;
          const V4 w4 = *(const V4*)(s_W + 4 * row);
          VT w[4] = {w4.x, w4.y, w4.z, w4.w};
          int j = 0;
          constexpr int UB = sizeof(VT) == 8 ? 2 : 4;
          for (; j + UB - 1 < nb; j += UB) {
            V4 av[UB];
#pragma unroll
            for (int u = 0; u < UB; ++u) av[u] = *(const V4*)(vbase + (size_t)(j + u) * Rcap * 4 + 4 * row);
#pragma unroll
            for (int u = 0; u < UB; ++u) {
              const VT v0[4] = {av[u].x, av[u].y, av[u].z, av[u].w};
              const VT* C0 = s_C + (j + u) * 16;
#pragma unroll
              for (int d = 0; d < 4; ++d) {
                VT t = w[d];
#pragma unroll
                for (int c = 0; c < 4; ++c) t -= v0[c] * (VT)C0[c * 4 + d];
                w[d] = t;
              }
            }
          }
          for (; j < nb; ++j) {
            const V4 a0 = *(const V4*)(vbase + (size_t)j * Rcap * 4 + 4 * row);
            const VT v0[4] = {a0.x, a0.y, a0.z, a0.w};
            const VT* C0 = s_C + j * 16;
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
        block_sum<10, LZ_NW>(acc, s_red, G);              // G[0..9] packed Gram
        bool again = false;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          const int dd = d == 0 ? 0 : (d == 1 ? 4 : (d == 2 ? 7 : 9));
          const double before = X[12 + d];
          if (s_flag[d] && before > tol * tol && G[dd] < 0.5 * before) again = true;
        }
        lds_barrier();                            // X, G read by all before reuse
        if (!again || pass == 1) break;
        ++n2;
      }
      // ---- 4. QR of W: one Cholesky QR when the factor is well conditioned
      // (pivot ratio > 1e-4, so kappa^2 eps < 1e-12), twice otherwise, and
      // modified Gram-Schmidt with deflation when a pivot is not safely > 0.
      // Without a re-orthogonalisation pass W is unchanged since step 3a,
      // whose factorisation of the same Gram matrix is used; after a pass
      // every thread factors the new Gram itself (no serial section).
      bool act[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) act[c] = s_flag[c] != 0;
      const int map[16] = {0, 1, 2, 3, 1, 4, 5, 6, 2, 5, 7, 8, 3, 6, 8, 9};
      if (g.scalar) {
        // orbital seeds: B_k = diag(|w_c|); a column whose norm is <= tol
        // ends its chain (its space is invariant)
        const int dg[4] = {0, 4, 7, 9};
        bool keep[4];
        double nrm[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          keep[c] = act[c] && G[dg[c]] > tol * tol;
          nrm[c] = keep[c] ? sqrt(G[dg[c]]) : 0.0;
        }
        lds_barrier();                              // every thread has read G
        if (tid == 0) {
#pragma unroll
          for (int q = 0; q < 16; ++q) { X[q] = 0.0; B[q] = 0.0; }
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            if (keep[c]) { B[c * 5] = nrm[c]; X[c * 5] = 1.0 / nrm[c]; }
            if (act[c] && !keep[c]) ++ndefl;
            s_flag[c] = keep[c] ? 1 : 0;
          }
          s_flag[5] = 0;
        }
        lds_barrier();
      } else if (reorth) {
        double Gf[16], Ur[16], Xr[16], ratio;
#pragma unroll
        for (int q = 0; q < 16; ++q) Gf[q] = G[map[q]];
        const bool ok = chol4r(Gf, act, Ur, tol * tol, ratio);
        inv_upper4r(Ur, act, Xr);
        lds_barrier();                              // every thread has read G
        if (tid == 0) {
#pragma unroll
          for (int q = 0; q < 16; ++q) { X[q] = Xr[q]; B[q] = Ur[q]; }
          s_flag[5] = !ok ? 2 : (ratio > 1e-4 ? 0 : 1);
        }
        lds_barrier();
      }
      const int path = s_flag[5];
      if (path == 1) {
        // second Cholesky QR: V = W U^-1 in place, Gram of V, refactor
        double acc[10];
#pragma unroll
        for (int q = 0; q < 10; ++q) acc[q] = 0.0;
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
        block_sum<10, LZ_NW>(acc, s_red, G);
        {
          double Gf[16], U2[16], X2[16], r2;
#pragma unroll
          for (int q = 0; q < 16; ++q) Gf[q] = G[map[q]];
          chol4r(Gf, act, U2, 0.0, r2);
          inv_upper4r(U2, act, X2);
          lds_barrier();                            // G, X, B read by all
          if (tid == 0) {
            double Bn[16];
#pragma unroll
            for (int r0 = 0; r0 < 4; ++r0)
#pragma unroll
              for (int c = 0; c < 4; ++c) {
                double sum = 0.0;
#pragma unroll
                for (int p = 0; p < 4; ++p) sum += U2[r0 * 4 + p] * B[p * 4 + c];
                Bn[r0 * 4 + c] = sum;
              }
#pragma unroll
            for (int q = 0; q < 16; ++q) { B[q] = Bn[q]; X[q] = X2[q]; }
          }
          lds_barrier();
        }
        ++n2;
      } else if (path == 2) {
        // modified Gram-Schmidt (twice) within the block, with deflation
        if (tid < 16) B[tid] = 0.0;
        lds_barrier();
        for (int c = 0; c < 4; ++c) {
          for (int ps = 0; ps < 2; ++ps) {
            for (int p = 0; p < c; ++p) {
              if (!s_flag[p]) continue;          // uniform (LDS)
              double a1[1] = {0.0};
              for (int row = tid; row < R; row += LZ_NT)
                a1[0] += (double)s_W[4 * row + p] * (double)s_W[4 * row + c];
              block_sum<1, LZ_NW>(a1, s_red, G);
              const double dot = G[0];
              for (int row = tid; row < R; row += LZ_NT)
                s_W[4 * row + c] = (VT)((double)s_W[4 * row + c] - dot * (double)s_W[4 * row + p]);
              if (tid == 0) B[p * 4 + c] += dot;
              lds_barrier();
            }
          }
          double a1[1] = {0.0};
          for (int row = tid; row < R; row += LZ_NT) a1[0] += (double)s_W[4 * row + c] * (double)s_W[4 * row + c];
          block_sum<1, LZ_NW>(a1, s_red, G);
          const double nrm = sqrt(G[0]);
          const bool keep = nrm > tol;
          const double sc = keep ? 1.0 / nrm : 0.0;
          for (int row = tid; row < R; row += LZ_NT) s_W[4 * row + c] = (VT)((double)s_W[4 * row + c] * sc);
          if (tid == 0) {
            if (keep) B[c * 4 + c] = nrm;
            else { for (int e = 0; e < 4; ++e) B[c * 4 + e] = 0.0; }
            if (s_flag[c] && !keep) ++ndefl;
            s_flag[c] = keep ? 1 : 0;
          }
          lds_barrier();
        }
        if (tid < 16) X[tid] = ((tid % 5) == 0) ? 1.0 : 0.0;
        lds_barrier();
      }
      // ---- 5. V_{k+1} = W X: LDS current block, HBM basis, J rows; B_k
      {
        VT* Vn = vbase + (size_t)(k + 1) * Rcap * 4;
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
          store4<VT>(s_Vo + 4 * row, v);             // V_{k+1}: the buffer of the next step
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
          if (g.ab_lds) s_ab[k * 32 + 16 + tid] = (float)B[tid];
          Bp[tid] = B[tid];
        }
        lds_barrier();
      }
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
      atomicAdd((unsigned long long*)&g.stats[ST_REORTH_STEPS], (unsigned long long)nreorth);
      atomicAdd((unsigned long long*)&g.stats[ST_BASIS_BYTES], (unsigned long long)bytes);
    }
    __syncthreads();
  }
}

size_t lanczos_lds_bytes(int nc_max, int r_max, bool fp32, int nt, bool om_lds, bool ab_lds, bool vprev_lds) {
  const size_t vt = fp32 ? 4 : 8;
  const size_t Rcap = 4 * (size_t)nc_max;
  const int nw = nt / 64;
  size_t b = 2 * Rcap * 4 * vt + 16;
  const int cslots = r_max > 2 * nw ? r_max : 2 * nw;
  b += (size_t)cslots * 16 * vt + 16 + nw * 16 * 8 + 224 * 8;
  b += (size_t)(nc_max + 1) * 4 + (size_t)nc_max * 4 + (size_t)nc_max * 2 + 16;
  if (om_lds) b += (size_t)3 * r_max * 16 * 4;
  if (ab_lds) b += (size_t)r_max * 32 * 4;
  if (vprev_lds) b += Rcap * 4 * vt + 16;
  return b + 64;
}

template <typename VT, bool BF = false, bool WIDE = false, bool MF = false, bool AL = false>
static void launch_lz(const LanczosArgs& a, int nt, int minw, int n_wg, size_t lds, hipStream_t st) {
  if (minw == 2) {
    if (nt == 256) hipLaunchKernelGGL((k_lanczos<VT, 256, 2, BF, WIDE, MF, AL>), dim3(n_wg), dim3(256), lds, st, a);
    else hipLaunchKernelGGL((k_lanczos<VT, 512, 2, BF, WIDE, MF, AL>), dim3(n_wg), dim3(512), lds, st, a);
  } else if (minw == 3) {                       // 256 threads only
    hipLaunchKernelGGL((k_lanczos<VT, 256, 3, BF, WIDE, MF, AL>), dim3(n_wg), dim3(256), lds, st, a);
  } else {
    if (nt == 256) hipLaunchKernelGGL((k_lanczos<VT, 256, 4, BF, WIDE, MF, AL>), dim3(n_wg), dim3(256), lds, st, a);
    else hipLaunchKernelGGL((k_lanczos<VT, 512, 4, BF, WIDE, MF, AL>), dim3(n_wg), dim3(512), lds, st, a);
  }
}

void launch_lanczos(const LanczosArgs& a, int precision, int nt, int minw, int layout, int n_wg, size_t lds,
                    hipStream_t st) {
  if (precision == TB_BF16) launch_lz<float, true>(a, nt, minw, n_wg, lds, st);
  else if (precision == TB_FP32 && layout == 3) launch_lz<float, false, false, false, true>(a, nt, minw, n_wg, lds, st);
  else if (precision == TB_FP32 && layout == 2) launch_lz<float, false, false, true>(a, nt, minw, n_wg, lds, st);
  else if (precision == TB_FP32 && layout == 1) launch_lz<float, false, true>(a, nt, minw, n_wg, lds, st);
  else if (precision == TB_FP32) launch_lz<float>(a, nt, minw, n_wg, lds, st);
  else if (layout == 3) launch_lz<double, false, false, false, true>(a, nt, minw, n_wg, lds, st);
  else launch_lz<double>(a, nt, minw, n_wg, lds, st);
}

hipError_t lanczos_set_lds(size_t lds) {
  const void* fn[35] = {(const void*)k_lanczos<double, 256, 4>, (const void*)k_lanczos<double, 512, 4>,
                        (const void*)k_lanczos<float, 256, 4>, (const void*)k_lanczos<float, 512, 4>,
                        (const void*)k_lanczos<double, 256, 2>, (const void*)k_lanczos<double, 512, 2>,
                        (const void*)k_lanczos<float, 256, 2>, (const void*)k_lanczos<float, 512, 2>,
                        (const void*)k_lanczos<float, 256, 4, true>, (const void*)k_lanczos<float, 512, 4, true>,
                        (const void*)k_lanczos<float, 256, 2, true>, (const void*)k_lanczos<float, 512, 2, true>,
                        (const void*)k_lanczos<float, 256, 4, false, true>, (const void*)k_lanczos<float, 512, 4, false, true>,
                        (const void*)k_lanczos<float, 256, 2, false, true>, (const void*)k_lanczos<float, 512, 2, false, true>,
                        (const void*)k_lanczos<double, 256, 3>, (const void*)k_lanczos<float, 256, 3>,
                        (const void*)k_lanczos<float, 256, 3, true>, (const void*)k_lanczos<float, 256, 3, false, true>,
                        (const void*)k_lanczos<float, 256, 4, false, false, true>,
                        (const void*)k_lanczos<float, 512, 4, false, false, true>,
                        (const void*)k_lanczos<float, 256, 2, false, false, true>,
                        (const void*)k_lanczos<float, 512, 2, false, false, true>,
                        (const void*)k_lanczos<float, 256, 3, false, false, true>,
                        (const void*)k_lanczos<float, 256, 4, false, false, false, true>,
                        (const void*)k_lanczos<float, 512, 4, false, false, false, true>,
                        (const void*)k_lanczos<float, 256, 2, false, false, false, true>,
                        (const void*)k_lanczos<float, 512, 2, false, false, false, true>,
                        (const void*)k_lanczos<float, 256, 3, false, false, false, true>,
                        (const void*)k_lanczos<double, 256, 4, false, false, false, true>,
                        (const void*)k_lanczos<double, 512, 4, false, false, false, true>,
                        (const void*)k_lanczos<double, 256, 2, false, false, false, true>,
                        (const void*)k_lanczos<double, 512, 2, false, false, false, true>,
                        (const void*)k_lanczos<double, 256, 3, false, false, false, true>};
  for (int q = 0; q < 35; ++q) {
    hipError_t e = hipFuncSetAttribute(fn[q], hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace tbk

