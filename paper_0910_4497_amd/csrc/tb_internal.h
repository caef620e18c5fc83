// Internal definitions shared by the HIP kernels and the host API of
// libtbkrylov. Device code is written for gfx950 (CDNA4, 64-lane waves).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "../../include/tbkrylov.h"

struct tb_ctx;

namespace tbk {

// BF16 (8 significand bits) by round-to-nearest-even of a finite FP32 value,
// returned as FP32.
__device__ __forceinline__ float bf16_round(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

constexpr int ZMAX_DEFAULT = 24;   // hop-list capacity of tb_create: neighbours within max(rm, dm)
constexpr int ZMAX_CAP = 256;      // largest hop-list capacity (tb_create_ex); rho rows = capacity + 1
constexpr int LOCAL_BITS = 11;     // local atom index bits in a packed coupling
constexpr int NCLUSTER_LIMIT = (1 << LOCAL_BITS) - 1;
constexpr int RMAX_LIMIT = 256;
constexpr int PROF_MAX = 4096;
constexpr int N_PHASES = 6;
constexpr size_t LDS_CU = 160 * 1024;   // LDS per compute unit (gfx950)
constexpr size_t LDS_RESERVE = 512;     // per workgroup: static LDS (a few bytes) and allocation rounding
constexpr int LZ_PER_CU_MAX = 4;   // Krylov workgroups per compute unit the tuner may pick
constexpr int EIG_PER_CU_MAX = 8;  // k_eig workgroups per compute unit the tuner may pick

// Device-side error / statistics words (int64 each).
enum StatSlot {
  ST_FLAGS = 0, ST_MAX_CLUSTER = 1, ST_MAX_HOP = 2, ST_MAX_COUPLINGS = 3,
  ST_DEFLATED = 4, ST_EARLY_STOP = 5, ST_MAX_CLUSTER_POS = 6, ST_MEMORY = 7,
  ST_REORTH2 = 8, ST_REORTH_STEPS = 9, ST_BASIS_BYTES = 10, ST_NSTATS = 16
};
enum FlagBits {
  FL_HOP_OVERFLOW = 1, FL_CLUSTER_OVERFLOW = 2, FL_COUPLING_OVERFLOW = 4,
  FL_NONFINITE = 8, FL_EIG_NOCONV = 16, FL_REFLOG_OVERFLOW = 32, FL_SEG_OVERFLOW = 64,
  FL_GROUP_IMAGE = 128
};

// Model parameters as the kernels see them (plain struct, passed by value).
struct Model {
  double eps_s, eps_p, v_sss, v_sps, v_pps, v_ppp;
  double r0, n, nc, rc, r1, rm, s_tail[4];
  double phi0, d0, m, mc, dc, d1, dm, phi_tail[4], frep[5];
};

struct Box {
  double L[3];
  int per[3];
};

constexpr int NCELL_AXIS_MAX = 64;   // cells per axis of the neighbour search
constexpr int GROUP_MAX = 8;          // atoms per group of the grouped form
constexpr int UNION_LDS_MAX = 8192;   // group members' sphere entries a union is built from (32 KiB)
struct CellGrid {
  int n[3];        // cells per axis (1 on a non-periodic axis)
  double len[3];   // cell edge (>= the cluster radius on a periodic axis with n > 1)
};

// --------------------------------------------------------------- helpers
__device__ __forceinline__ double mic(double d, double L, int per) {
  return per ? d - L * rint(d / L) : d;
}

// Xu-form scaled function pre * (r0/r)^ex * exp{ex[-(r/rc)^exc + (r0/rc)^exc]}
// below r1, cubic tail on [r1, rmax), zero beyond; value and r-derivative.
__device__ __forceinline__ void xu_radial(double r, double pre, double r0, double ex,
                                          double exc, double rc, double r1, double rmax,
                                          const double* tail, double& val, double& dval) {
  if (r >= rmax) { val = 0.0; dval = 0.0; return; }
  if (r >= r1) {
    double x = r - r1;
    val = tail[0] + x * (tail[1] + x * (tail[2] + x * tail[3]));
    dval = tail[1] + x * (2.0 * tail[2] + x * 3.0 * tail[3]);
    return;
  }
  double q = pow(r / rc, exc);
  double q0 = pow(r0 / rc, exc);
  val = pre * pow(r0 / r, ex) * exp(ex * (q0 - q));
  dval = val * (-ex / r) * (1.0 + exc * q);
}

__device__ __forceinline__ void hop_scale(const Model& M, double r, double& s, double& ds) {
  xu_radial(r, 1.0, M.r0, M.n, M.nc, M.rc, M.r1, M.rm, M.s_tail, s, ds);
}

__device__ __forceinline__ void pair_term(const Model& M, double r, double& phi, double& dphi) {
  xu_radial(r, M.phi0, M.d0, M.m, M.mc, M.dc, M.d1, M.dm, M.phi_tail, phi, dphi);
}

// 64-lane wave reductions through cross-lane shuffles.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
// Workgroup barrier that orders LDS only. Unlike __syncthreads() it does not
// wait for the thread's outstanding global stores; use it where no other
// thread of the workgroup reads those stores before a later full barrier.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
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

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}


// ------------------------------------------------------------ kernel args
struct LanczosArgs {
  int atom0, n_atoms, r_default;       // target atoms [atom0, n_atoms) of this launch
  const int* r_per_atom;
  const int* clu_n; const int* clu_j; const int* loc_off; const uint32_t* loc_ent;
  int zmax;                    // hop-list capacity (rho rows per target: zmax + 1)
  const double* hnorm; const int* jloc; const int* hop_n;
  const void* pair;            // [N][zmax][4] double or float: hx hy hz s
  int nc_max; int64_t emax; int r_max;
  double eps_s, eps_p, v_sss, v_sps, v_pps, v_ppp;
  void* vbuf;                  // [WG][r_max][4*nc_max][4]
  double* tab;                 // [N][r_max][2][16]: A_k, B_k
  int* kused;
  void* vj;                    // [N][4*(zmax+1)][4*r_max]
  int* counter;
  double* omega;               // [WG][3][r_max][16] float orthogonality estimates (when not in LDS)
  int om_lds;                  // estimates kept in LDS
  int ab_lds;                  // FP32 copies of A_j, B_j kept in LDS (needs om_lds)
  int vprev_lds;               // V_{k-1} kept in a second LDS block buffer
  int scalar;                  // orbital seeds: four independent scalar chains (diagonal A_k, B_k)
  double eta, eps_unit;        // re-orthogonalisation threshold, unit roundoff of VT
  int64_t* stats;
};
size_t lanczos_lds_bytes(int nc_max, int r_max, bool fp32, int nt, bool om_lds, bool ab_lds, bool vprev_lds);
// precision: TB_FP64 / TB_FP32 / TB_BF16; nt: 256 or 512 threads; minw: 2, 3
// (256 threads only) or 4 waves per SIMD (register budget)
// layout: 0 one column per lane (FP32, BF16) or four lanes per atom (FP64);
// FP32 only: 1 the four-columns-per-lane H.V items, 2 the MFMA items; FP32 and
// FP64: 3 one target atom per lane (see k_lanczos)
void launch_lanczos(const LanczosArgs& a, int precision, int nt, int minw, int layout, int n_wg, size_t lds,
                    hipStream_t st);
hipError_t lanczos_set_lds(size_t lds);

struct EigArgs {
  int atom0, n_atoms, r_max;           // target atoms [atom0, n_atoms) of this launch
  const double* tab; const int* kused;
  double* lam; double* wgt; double* y1;
  double* ref_v; uint16_t* ref_p; int* ref_n; int64_t ref_max;   // band reduction's reflector log
  int* seg; int* seg_n; int seg_max;   // [N][seg_max] segment starts; [N][2]: segment counts
  int* counter;                        // persistent-kernel atom queue (zeroed before launch)
  double* scratch;                     // [WG][4 r_max][4][threads]: LU factors of inverse iteration
  void* evec;                          // [N][4 r_max][4 r_max]: eigenvectors of the tridiagonal, column t at t * 4 r_max
  int u_fp32;                          // evec holds float (after the FP32 recursion) or double
  double* vsc;                         // [N][4 r_max]: factor that normalises column t of evec
  double* tri;                         // [N][2][4 r_max]: diagonal and off-diagonal of the tridiagonal
  int64_t* stats;
  int scalar;                          // orbital seeds: T is four independent chains (k_eig_chains)
};
struct RhoArgs {
  int atom0, n_atoms, r_max;           // target atoms [atom0, n_atoms) of this launch
  const int* kused; const int* hop_n; const int* clu_j; int nc_max;
  int zmax;                            // hop-list capacity (rho rows per target: zmax + 1)
  const double* lam; const double* y1;
  const double* ref_v; const uint16_t* ref_p; const int* ref_n; int64_t ref_max;
  const int* seg; const int* seg_n; int seg_max;
  const void* evec; const double* vsc;     // evec: float when vj_fp32, else double
  const void* vj; int vj_fp32;
  const int64_t* row_ptr;
  const double* mu_state; double kT;
  double* rho;
  int64_t* stats;
};
size_t eig_lds_bytes(int r_max);
int64_t band_reflectors(int d);     // reflectors of the band reduction of a d x d T
int band_segments(int d);           // replay segments of that reduction
size_t rho_lds_bytes(int r_max);
hipError_t eig_set_lds(int r_max);
void launch_eig(const EigArgs& a, int n_wg, hipStream_t st);
int eig_threads(int r_max);
void launch_rho(const RhoArgs& a, hipStream_t st);

struct MuArgs {
  int64_t n_pairs;             // atoms * 4 r_max (padding has w = 0)
  const double* lam; const double* wgt;
  double kT, n_e;
  double* state;               // [mu_state_doubles()]: [2] the final mu, then two bracket states
  double* partial;             // [mu_partial_doubles()]: per-block partial sums, three regions
  double* eparts; double* mu_out;
};
int mu_blocks(int64_t n_pairs);
size_t mu_partial_doubles();
size_t mu_state_doubles();
void launch_mu(const MuArgs& a, double mu_fixed, bool fixed, int n_iter, hipStream_t st);

struct ForceArgs {
  int n_atoms, zmax;
  Model M;
  const int* hop_n; const int* hop_j; const int* hop_rev; const double* hop_d;
  const int64_t* row_ptr;
  const double* rho;          // [pairs][4][4]: rho[p][a][b] = rho_{j a, i b}
  double* xrep;               // [N][2]: F'(x_i), F(x_i)
  double* forces;             // [N][3] (nullable)
  const double* grad_scale;   // nullable: forces receive -(*grad_scale) F (the backward of E_tot)
  double* eparts; double kT;
  double* e_out;              // [4] (nullable in the backward)
  double* wpart;              // [blocks][9] per-block virial sums
  double* virial;             // [9] W[a][b] = sum over ordered pairs of d_a g_b
};
void launch_forces(const ForceArgs& a, bool with_forces, hipStream_t st);
// Fixed device workspace of tb_energy_forces_static (a file-scope array of
// tb_forces.hip): its address on `device` (current) is looked up once by
// static_scratch_init; static_scratch_args points xrep and wpart into it
// (false before the lookup); static_scratch_need is the size for n atoms.
hipError_t static_scratch_init(int device);
bool static_scratch_args(int device, ForceArgs& a);
size_t static_scratch_need(int64_t n_atoms);
size_t static_scratch_bytes();
void launch_virial_copy(const double* src, double* dst, hipStream_t st);

// K1-K3 and the rho pair layout for the geometry in pos (device).
void launch_build(tb_ctx* c, const double* pos, double r_list, hipStream_t st);

}  // namespace tbk

// Context (host struct; all pointers are device memory unless noted).
struct tb_ctx {
  int device;
  hipStream_t stream;
  int64_t na_max;
  int nc_max, r_max;
  int64_t emax;          // couplings per sphere
  int64_t ref_max;       // reflector-log entries per atom
  int n_cu;              // compute units of the device
  // launch shape of the Krylov kernel per precision ([0] FP64, [1] FP32, [2] BF16):
  // threads per workgroup, register budget (waves per SIMD) and persistent
  // workgroups per compute unit
  int lz_nt[3], lz_minw[3], lz_per_cu[3], lz_wide[3];
  int lz_per_cu_max;     // workspace is sized for this many per compute unit
  int eig_per_cu, eig_per_cu_max;   // persistent k_eig workgroups per compute unit
  int atoms_per_launch;  // 0: one launch per phase; k: per-atom phases in launches of k atoms
  int seeds;             // TB_SEEDS_BLOCK or TB_SEEDS_ORBITAL
  int group_m;           // atoms per group of the grouped form (union spheres); 0 or 1: own spheres
  size_t bytes;

  // state
  int stage;             // 0 none, 1 lists built, 2 rho built
  int64_t n_atoms;
  tbk::Model model;
  tbk::Box box;
  double r_cluster;
  double kT;
  int precision;
  int64_t nnz_pairs;     // host copy (valid after tb_rho_layout)
  const double* rho_last; // rho_out of the last tb_krylov_rho

  // lists (K1-K3)
  int zmax;                                                // hop-list capacity
  int* hop_n; int* hop_j; int* hop_rev; double* hop_d;     // [N][zmax][4]: dx dy dz r
  double* pair64; float* pair32;                           // [N][zmax][4]: hx hy hz s
  int* clu_n; int* clu_j;                                  // [N][NC]
  int* cell_of; int* cell_atoms;                           // [N]: cell of each atom, atoms by cell
  int* cell_cnt; int* cell_start;                          // [CELLS], [CELLS + 1]
  int* loc_off; uint32_t* loc_ent;                         // [N][NC+1], [N][EMAX]: b | slot << LOCAL_BITS
  double* hnorm;                                           // [N]
  int* jloc;                                               // [N][zmax + 1]
  int64_t* row_ptr;                                        // [N+1]
  int* col_j;                                              // [N*(zmax + 1)] (pairs, compact)
  // Krylov (K4)
  void* vbuf;            // [WG][RMAX][4*NC][4] f64 or f32
  double* omega;         // [WG][3][RMAX][16] orthogonality estimates
  double* tab;           // [N][RMAX][2][16]
  int* kused;            // [N]
  void* vj;              // [N][4*(zmax + 1)][4*RMAX] f64 or f32
  int* work_counter;     // persistent-kernel atom queue
  // eigen (K5/K7)
  double* lam; double* wgt; double* y1;                    // [N][D], [N][D], [N][4][D]
  double* ref_v; uint16_t* ref_p; int* ref_n;             // [N][REF][4] (v1 v2 v3 tau), [N][REF] (row), [N]
  int* seg; int* seg_n; int seg_max;                       // [N][SEG], [N][2]
  double* evec;                                            // [N][D][D], column by column
  double* vsc;                                             // [N][D] normalising factors of the evec columns
  double* tri;                                             // [N][2][D]
  double* eig_scratch;                                     // [WG_EIG][D][4][EIG_NT]
  // mu / energies (K6/K8)
  double* mu_state;      // [2]: mu; [16..47]: two multisection states
  double* partial;       // per-block partial sums of the mu reductions
  double* xrep;          // [N]: sum_j phi, then F'(x)
  double* eparts;        // [4] band, entropy, rep, count
  double* wpart;         // [ceil(N/64)][9] per-block virial sums
  double* virial;        // [9] virial of the last tb_energy_forces
  int have_virial;       // tb_energy_forces ran on the current rho
  int64_t* stats;        // [ST_NSTATS]
  // phase timing
  int prof;
  hipEvent_t* ev_pool;   // [2 * PROF_MAX]
  int* ev_phase;         // host [PROF_MAX]
  int ev_used;
  int64_t ev_dropped;
};
