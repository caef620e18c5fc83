/*
 * libtbkrylov -- local Krylov-subspace density-matrix solve for linear-scaling
 * tight-binding molecular dynamics on AMD Instinct MI355X (gfx950).
 *
 * The method (Iitaka, "GPU-accelerated large-scale quantum molecular dynamics
 * simulation of 3-dimensional C60 polymers"):
 *   - Sec. 2, Eq. (1): a non-self-consistent tight-binding Hamiltonian with
 *     on-site energies and two-centre hoppings; here an orthogonal sp3
 *     Slater-Koster model, orbitals (s, px, py, pz) on every atom.
 *   - Sec. 2, Eq. (2): the one-body density matrix rho = sum_m |m> f(e_m) <m|,
 *     forces <F_i> = Tr[rho F_i] with F_i = -dH/dR_i.
 *   - Sec. 2 (locality): every target atom i is solved using only the atoms
 *     inside a cutoff sphere of radius r_cluster around it (cost O(n^3 N)).
 *   - Sec. 3, Eq. (4): that local problem is projected on the Krylov subspace
 *     K_r(H, Phi_i) = span{Phi_i, H Phi_i, ..., H^{r-1} Phi_i} seeded with the
 *     target atom's orbitals (here all four of them, as one seed block), built
 *     by the Lanczos recursion of Eqs. (6)-(9) in block form; the projected
 *     block-tridiagonal matrix is diagonalised (Sec. 3, the LAPACK step).
 *
 * Conventions
 *   - Every function returns an int status: TB_OK (0) or a negative TB_E* code;
 *     tb_last_error() then holds a message.
 *   - Pointers are DEVICE pointers unless their name ends in _host.
 *   - Arrays are row-major (C order). Units: Angstrom, eV, eV/Angstrom.
 *   - All work is enqueued on the stream given to tb_create; no function
 *     synchronises the stream implicitly except tb_rho_layout (it returns a
 *     host count) and tb_get_stats. Outputs are valid after a stream sync.
 *   - The caller owns every input and output buffer. The context owns every
 *     work buffer (neighbour and cluster lists, Hamiltonian pair data, Krylov
 *     bases, projected matrices, eigen data, the chemical potential); it sizes
 *     them once in tb_create from the capacities given there.
 *   - Call order per geometry: tb_build_local_H -> tb_krylov_rho ->
 *     tb_energy_forces. A call out of order returns TB_ESTATE.
 */
#ifndef TBKRYLOV_H
#define TBKRYLOV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  TB_OK = 0,
  TB_EINVAL = -1,       /* null, non-finite or out-of-range argument */
  TB_ECUTOFF = -2,      /* cutoff >= half a periodic box length */
  TB_ECAPACITY = -3,    /* a list or Krylov size exceeds the tb_create capacity */
  TB_EMU = -4,          /* electron count outside (0, 8N) */
  TB_EUNSUPPORTED = -5, /* feature not provided (e.g. a non-orthorhombic cell) */
  TB_EHIP = -6,         /* HIP runtime error; message holds the HIP error text */
  TB_ESTATE = -7,       /* functions called out of order */
  TB_EDEVICE = -8       /* a kernel raised its error flag (see tb_get_stats) */
};

/* Precision of the Krylov recursion (H.V products, basis storage and the
 * re-orthogonalisation). Projected eigensolve, chemical potential, block
 * normalisation norms, density-matrix assembly and forces are FP64 always.
 *   TB_FP64  everything in FP64.
 *   TB_FP32  H.V, basis, three-term update and passes in FP32 (norms and
 *            Gram sums accumulated in FP64).
 *   TB_BF16  as TB_FP32, but the V_k operand of H.V is rounded to BF16 (the
 *            Hamiltonian -- on-site and bond parameters, pair data -- stays
 *            FP32) and the products accumulated in FP32; the orthogonality
 *            estimate then asks for a re-orthogonalisation pass at every
 *            block step. Its force error is far above 1e-3 eV/A: measured,
 *            not a production mode. */
enum { TB_FP64 = 0, TB_FP32 = 1, TB_BF16 = 2 };

/* Tight-binding parameters of the Xu-form carbon model (Sec. 4 names the
 * Xu parameter set, cutoff 2.6 A). Hopping scale s(r) = (r0/r)^n
 * exp{n[-(r/rc)^nc + (r0/rc)^nc]} below r1, the cubic
 * s_tail[0] + s_tail[1] x + s_tail[2] x^2 + s_tail[3] x^3 (x = r - r1) on
 * [r1, rm), zero beyond rm. The pair term phi(r) has the same form with
 * (phi0, d0, m, mc, dc, d1, dm, phi_tail); E_rep = sum_i F(sum_j phi(r_ij)),
 * F(x) = sum_k frep[k] x^k. struct_size must equal sizeof(tb_params). */
typedef struct {
  int64_t struct_size;
  double eps_s, eps_p, v_sss, v_sps, v_pps, v_ppp; /* eV */
  double r0, n, nc, rc, r1, rm, s_tail[4];
  double phi0, d0, m, mc, dc, d1, dm, phi_tail[4], frep[5];
} tb_params;

typedef struct tb_ctx tb_ctx;

/* Create a context on HIP device `hip_device`, enqueuing on `hip_stream`
 * (a hipStream_t, or NULL for the default stream). The capacities are the
 * sizes of the paper's problem: at most n_atoms_max atoms (N, Sec. 2),
 * n_cluster_max atoms per cutoff sphere (n, the sphere of the locality
 * argument of Sec. 2 whose cost is O(n^3 N)), r_max Krylov block steps (the
 * order r of K_r in Sec. 3, Eq. 4); hop lists hold at most 24 neighbours
 * within max(rm, dm) (the 2.6 A hopping range of Xu's parameters, Sec. 4;
 * tb_create_ex sets another capacity). The context owns every work buffer
 * sized from these; *ctx receives it (NULL on error).
 * Allocates all work memory (size reported by tb_get_stats) and synchronises
 * the device once; no later call allocates device memory.
 * Errors: TB_EINVAL (null ctx pointer, a capacity outside its range: n_atoms_max
 * in [1, 2^24], n_cluster_max in [1, 2047], r_max in [1, 256], or no such
 * device), TB_ECAPACITY (a sphere of n_cluster_max atoms or r_max steps do
 * not fit a compute unit's LDS), TB_EHIP (allocation failed). */
int tb_create(tb_ctx **ctx, int hip_device, void *hip_stream,
              int64_t n_atoms_max, int n_cluster_max, int r_max);

/* tb_create with a hop-list capacity of hop_max neighbours within max(rm, dm)
 * per atom (1 <= hop_max <= 256): hopping ranges longer than the 2.6 A of
 * Xu's set, such as the 7 A interlayer range of the paper's second
 * parameter set (Sec. 4), need ~200. The density-matrix blocks of a target
 * are its hop list plus itself, so rho_out needs room for
 * n_atoms * (hop_max + 1) blocks. tb_create is tb_create_ex with 24.
 * Errors: as tb_create, and TB_EINVAL for hop_max outside [1, 256]. */
int tb_create_ex(tb_ctx **ctx, int hip_device, void *hip_stream,
                 int64_t n_atoms_max, int n_cluster_max, int r_max, int hop_max);

/* Release a context and all its work memory (the buffers of the problem of
 * Secs. 2-3 that tb_create sized). Waits for nothing: the caller must have
 * synchronised the context's stream first, since enqueued kernels still read
 * the work buffers. NULL is accepted (no-op). Returns TB_OK. */
int tb_destroy(tb_ctx *ctx);

/* Sec. 2 locality + Eq. (1): minimum-image neighbour lists, cutoff spheres
 * C_i = {i} + {j : |d_ij| < r_cluster} (sorted by j), Slater-Koster pair data
 * for every ordered pair closer than rm, and each sphere's local block
 * structure. Two atoms a, b of C_i are coupled iff |x_b - x_a| < rm, where x
 * is the position relative to the target atom i (minimum image).
 *   pos       [n_atoms][3] device, Angstrom.
 *   cell_host [3][3] row vectors of an orthorhombic box (off-diagonals 0).
 *   periodic_host[3] 0/1 per axis; a non-periodic axis ignores the box.
 * n_cluster_out [n_atoms] (device, nullable) receives |C_i|.
 * Errors: TB_EINVAL, TB_ECUTOFF (r_cluster or rm >= half a periodic box
 * length), TB_EUNSUPPORTED (non-orthorhombic), TB_ECAPACITY (raised on the
 * next call from the device flag when a list overflows). */
int tb_build_local_H(tb_ctx *ctx, int64_t n_atoms, const double *pos,
                     const double *cell_host, const int *periodic_host,
                     const tb_params *p_host, double r_cluster,
                     int *n_cluster_out);

/* Sec. 3: for every target atom, r block steps of the block Lanczos
 * recursion (Eqs. 6-9 with 4x4 blocks A_k, B_k, seed = the atom's four
 * orbitals), the eigensolve of the projected block-tridiagonal T, the global
 * chemical potential and the density-matrix blocks of Eq. (2) restricted to
 * the Krylov space. The basis is kept orthogonal by partial
 * re-orthogonalisation: a running estimate of |V_j^T V_{k+1}| (the block form
 * of Simon's recurrence) triggers a full Gram-Schmidt pass against all
 * earlier blocks, for that block and the next, whenever it exceeds 1e-12
 * (TB_FP64) or 1e-4 (TB_FP32), so the result is the projection on K_r to
 * that level:
 *     rho[:, i] = Q Y f(Lambda) Y[0:4, :]^T,  f(e) = 2 / (1 + exp((e - mu)/kT)).
 *   r           block steps (1 <= r <= r_max) unless r_per_atom is given.
 *   r_per_atom  [n_atoms] device int, nullable: per-atom r.
 *   mu          fixed chemical potential in eV, or NaN: then mu solves
 *               sum_i sum_m f(lambda_m^i) w_m^i = n_electrons
 *               (w_m^i = weight of Ritz pair m on the seed block).
 *   precision   TB_FP64, TB_FP32 or TB_BF16 (see the enum).
 *   mu_out      device double (nullable) receives mu.
 *   rho_out     [nnz_pairs][4][4] device: rho_out[p][a][b] = rho_{j a, i b}
 *               for the pair list of tb_rho_layout (target i, row atom j).
 * Errors: TB_EINVAL, TB_ECAPACITY, TB_EMU, TB_ESTATE. */
int tb_krylov_rho(tb_ctx *ctx, int r, const int *r_per_atom, double kT,
                  double mu, double n_electrons, int precision,
                  double *mu_out, double *rho_out);

/* Pair list of rho_out. The density matrix of Eq. (2) is needed only on the
 * sparsity pattern of H (Eq. 1), because the forces Tr[rho F_i] of Sec. 2
 * contract it with dH/dR, which vanishes beyond the hopping range: for target
 * atom i (the column block rho_{., i} of its Krylov solve), the rows row_ptr[i]
 * .. row_ptr[i+1]-1 hold j = i first, then the atoms closer than max(rm, dm)
 * to i (the hop list) in increasing index. nnz_pairs_host receives the count
 * (host, required). row_ptr [n_atoms+1] (int64) and col_j [nnz] are device
 * arrays owned by the caller (nullable: count only).
 * Synchronises the stream. Valid after tb_build_local_H.
 * Errors: TB_EINVAL (null ctx or nnz_pairs_host), TB_ESTATE (no
 * tb_build_local_H yet), TB_EHIP. */
int tb_rho_layout(tb_ctx *ctx, int64_t *nnz_pairs_host, int64_t *row_ptr,
                  int *col_j);

/* Sec. 2: band energy, entropy term, repulsion and forces from the density
 * blocks of the last tb_krylov_rho:
 *   E_band = sum_i sum_m lambda_m f_m w_m,
 *   -TS    = -kT sum_i sum_m w_m 2 s(f_m/2),  s(q) = -q ln q - (1-q) ln(1-q),
 *   E_rep  = sum_i F(sum_j phi(r_ij)),
 *   F_k    = -sum_i sum_{j in hop(i)} Tr[(dH_ij/dR_k) rho_ji] - dE_rep/dR_k.
 *   e_out  [4] device: E_band, -TS, E_rep, E_tot = E_band - TS + E_rep (eV).
 *   forces [n_atoms][3] device, eV/Angstrom (nullable: energies only, and the
 *          force and virial contraction is not run; tb_virial then refuses).
 * Errors: TB_EINVAL (null ctx or e_out), TB_ESTATE, TB_EHIP. */
int tb_energy_forces(tb_ctx *ctx, double *e_out, double *forces);

/* tb_energy_forces for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels, the same results bit for bit, with their
 * partial results (per-atom repulsion staging, 16 B per atom, and per-block
 * virial sums, 72 B per 64 atoms) in a fixed 2 MiB device array of the
 * library instead of the context's workspace; it calls no allocating
 * routine. The array's address on each device is looked up when the first
 * context is created there. At most about 122,000 atoms (static_scratch_need
 * <= 2 MiB). All calls on one device share the array: calls that overlap
 * on one device (other streams, other contexts, other threads) race, so
 * serialise them. Arguments and outputs as tb_energy_forces.
 * Errors: TB_EINVAL, TB_ESTATE, TB_ECAPACITY (too many atoms for the
 * array), TB_EHIP. */
int tb_energy_forces_static(tb_ctx *ctx, double *e_out, double *forces);

/* Backward of the total energy E_tot = E_band - TS + E_rep of the last
 * tb_krylov_rho (Sec. 2: the force on an atom is Tr[rho F_i] with
 * F_i = -dH/dR_i, plus the repulsive term): with g = *grad_e (a device
 * scalar, the gradient flowing into E_tot),
 *   grad_pos[k] = -g * F_k,  F_k = -sum_i sum_{j in hop(i)} Tr[(dH_ij/dR_k) rho_ji] - dE_rep/dR_k,
 * the force contraction of tb_energy_forces scaled by g in the same kernel.
 * At finite r and cutoff F is the method's force, not the exact gradient of
 * E_tot (the local density matrix is not variational).
 *   grad_e   device double (the upstream gradient).
 *   grad_pos [n_atoms][3] device, eV/Angstrom times the unit of g.
 * Also refreshes the virial (tb_virial). Enqueued on the stream.
 * Errors: TB_EINVAL (null pointer), TB_ESTATE (no tb_krylov_rho yet). */
int tb_energy_backward(tb_ctx *ctx, const double *grad_e, double *grad_pos);

/* Virial of the last tb_energy_forces (Sec. 5 times the pressure of a diamond
 * cell; Sec. 4 compresses the C60 crystal). With d_ij = R_j - R_i (minimum
 * image) and g_ij the derivative with respect to d_ij of the pair's energy
 * terms that the forces sum (Tr[H_ij rho_ji] of seed i, and the embedding
 * term F'(x_i) phi'(r_ij) d_ij / r_ij):
 *   W[a][b] = sum over ordered pairs (i, j) of (d_ij)_a (g_ij)_b  (eV).
 * Stress sigma = W / V, pressure P = -(W[0][0] + W[1][1] + W[2][2]) / (3 V);
 * for an isolated system W = -sum_k R_k (x) F_k. Like the forces, at finite r
 * and cutoff this is the method's virial, not the exact strain derivative of
 * E_tot. virial_out: device [3][3] row-major. Enqueued on the stream (no
 * synchronisation); the sums run in a fixed order (bitwise reproducible).
 * Errors: TB_EINVAL, TB_ESTATE (tb_energy_forces not called on this rho). */
int tb_virial(tb_ctx *ctx, double *virial_out);

/* Seeding of the Krylov spaces (Sec. 3). TB_SEEDS_BLOCK (the default): the
 * four orbitals of the target atom form one seed block, K_r = span{Phi,
 * H Phi, ..., H^{r-1} Phi}, block recursion with full 4x4 A_k and
 * upper-triangular B_k. TB_SEEDS_ORBITAL: the paper's own seeding, one scalar
 * Krylov space K_r(H, |i alpha>) per orbital alpha (Eq. 4 with the orbital as
 * seed), the four chains run together with diagonal A_k, B_k (Eqs. 8-9),
 * each re-orthogonalised against its own vectors only; the density-matrix
 * column of orbital alpha comes from its own chain. The orbital form is not
 * invariant under rotations of the atoms at finite r (the block form is), and
 * needs r up to the grade of each orbital (~4x the block order) to reach the
 * exact limit. Host-side setting; applies to later tb_krylov_rho calls.
 * Errors: TB_EINVAL. */
enum { TB_SEEDS_BLOCK = 0, TB_SEEDS_ORBITAL = 1 };
int tb_set_seeds(tb_ctx *ctx, int seeds);

/* Grouped form (Sec. 3): the atoms are taken in groups of m consecutive
 * indices {g m, ..., g m + m - 1} (the last group ragged), and the m atoms of
 * a group run their recursions on one Hamiltonian, that of the union of the
 * group's cutoff spheres: for every member i the sphere becomes
 *     C_G(i) = {i} + {j != i : min over members k of |d_kj| < r_cluster},
 * sorted by j, with positions relative to i (minimum image). With
 * TB_SEEDS_ORBITAL this is the paper's form, 4m scalar chains with diagonal
 * A_k, B_k per group; with TB_SEEDS_BLOCK each member's seed block runs on
 * the union sphere. m = 1 (the default) is each atom's own sphere. Callers
 * order the atoms so that a group's members are close (atoms of one molecule
 * consecutive, or a spatial sort); n_cluster_max must hold the union spheres.
 * Every member must satisfy |(d_ik)_a| + r_cluster < L_a / 2 on each periodic
 * axis a (unique images); otherwise the next tb_get_stats returns
 * TB_ECUTOFF. Host-side setting: the next tb_build_local_H builds the
 * unions (one workgroup per group, sort and unique in LDS), and until then
 * the context counts as not built.
 * Errors: TB_EINVAL (m outside [1, 8]), TB_ECAPACITY (m * n_cluster_max
 * > 8192). */
int tb_set_groups(tb_ctx *ctx, int m);

/* Launch granularity of the per-atom phases of tb_krylov_rho (block Lanczos,
 * projected eigensolve, density-matrix assembly). Every target atom's local
 * solve is independent once the couplings are built (Sec. 2, the cutoff
 * sphere): atoms_per_launch = 0 (the default) runs each phase as one launch
 * over all atoms; k >= 1 runs it as consecutive launches over groups of k
 * atoms (k = 1: one launch per atom), each with at most k workgroups. The
 * results are bitwise the same in every mode; only the launch count and the
 * device occupancy change. Host-side setting, no device work.
 * Errors: TB_EINVAL (ctx null or atoms_per_launch < 0). */
int tb_set_launch(tb_ctx *ctx, int atoms_per_launch);

/* Launch-shape autotuner for tb_krylov_rho at this precision. On the spheres
 * of the last tb_build_local_H (required first), it times the block-Lanczos
 * kernel for every launch shape that fits the device (256 or 512 threads per
 * workgroup x a register budget of 128 or 256 VGPRs x 1..4 persistent
 * workgroups per compute unit that stay co-resident, with as many of the
 * recursion's side buffers in LDS as that occupancy leaves room for), and
 * then the projected eigensolver for 2..8 persistent workgroups per compute
 * unit; every candidate runs twice, the faster run counts, and the fastest
 * shapes are kept in the context for later calls at this precision. Shapes
 * change launch geometry, registers and LDS residency, and with the thread
 * count the order of the workgroup reductions: later results agree with
 * those of the default shape to rounding (FP64: ~1e-15 relative). r, r_per_atom: as for
 * tb_krylov_rho. shape_out (host, nullable) [6]: Krylov threads per
 * workgroup, Krylov workgroups per compute unit, eigensolver workgroups per
 * compute unit, candidates timed, Krylov waves per SIMD of the register
 * budget (4: 128 VGPRs, 2: 256), and the layout of the H.V work items
 * (TB_FP32: 0 one column per lane; 1 four columns per lane over every
 * fourth coupling, which loads each coupling once; 2 the 4x4 Slater-Koster
 * blocks times the 4x4 blocks of V_k on the matrix cores, 16 target atoms per
 * wave; 3 one target atom per lane with all four columns in registers; all
 * four are timed. TB_FP64: 0 the four-lanes-per-atom items of layout 1, or
 * 3; both timed. TB_BF16: 0).
 * Synchronises the stream (not for graph
 * capture); tb_krylov_rho must run again before tb_energy_forces, and the
 * counters of tb_get_stats are those of before the call.
 * Errors: TB_EINVAL, TB_ESTATE, TB_ECAPACITY (r > r_max), TB_EHIP. */
int tb_autotune(tb_ctx *ctx, int r, const int *r_per_atom, int precision, int *shape_out);

/* Fixes the Krylov launch shape of later tb_krylov_rho calls at `precision`
 * without timing (the shapes tb_autotune chooses among): threads per
 * workgroup (256 or 512), waves per SIMD of the register budget (4: 128
 * VGPRs, 3: 168, with 256 threads only, 2: 256), persistent workgroups per
 * compute unit (they must stay
 * co-resident: wg_per_cu * threads / 64 <= 4 * waves_per_simd, and the
 * sphere capacity must fit their LDS) and the H.V item layout (wide = 0:
 * one column per lane for TB_FP32 and TB_BF16, four lanes per atom for
 * TB_FP64; 1, TB_FP32 only: four columns per lane over every fourth
 * coupling; 2, TB_FP32 only: the 4x4 blocks of 16 target atoms per wave on
 * the matrix cores, v_mfma_f32_4x4x1_16b_f32, one coupling slot per four
 * MFMAs; 3, TB_FP32 and TB_FP64: one target atom per lane, all four columns
 * over all of its couplings). Results of
 * different shapes agree to rounding; one shape gives the same bits on every
 * run. Host-side setting, no device work.
 * Errors: TB_EINVAL (a value outside those sets), TB_ECAPACITY (the LDS
 * of the workgroups does not fit a compute unit). */
int tb_set_shape(tb_ctx *ctx, int precision, int threads, int waves_per_simd, int wg_per_cu, int wide);

/* Diagnostics (host): counters since the last tb_build_local_H. stats_host
 * receives up to n_stats values: [0] device error flags, [1] max cluster
 * size, [2] max hop count, [3] max local couplings per sphere, [4] total
 * deflated columns, [5] atoms whose recursion stopped early (invariant
 * space), [6] largest eigenvalue-cluster position (0: no clusters), [7] work
 * memory bytes, [8] re-orthogonalisation second passes, [9] block steps
 * with a re-orthogonalisation pass, [10] basis bytes the Krylov kernel
 * moved (blocks written, read by the recursion and by the passes).
 * Synchronises the stream. */
int tb_get_stats(tb_ctx *ctx, int64_t *stats_host, int n_stats);

/* Per-phase timing with HIP events recorded on the context stream.
 * tb_profile_enable(ctx, 1) starts recording start/end events around each
 * phase (0: lists + local structure, 1: block Lanczos, 2: projected
 * eigensolve, 3: chemical potential, 4: density-matrix assembly, 5: energy
 * and forces); 0 stops. tb_profile_read synchronises the stream, adds the
 * elapsed times of all recorded phases into ms_host[phase] and their launch
 * counts into count_host[phase] (arrays of n >= 6), and clears the record.
 * At most 4096 phase records are kept between reads; further ones are
 * dropped and counted in count_host[6] if n > 6. */
int tb_profile_enable(tb_ctx *ctx, int enable);
int tb_profile_read(tb_ctx *ctx, double *ms_host, int64_t *count_host, int n);

/* Message for the last nonzero status returned on the calling thread: which
 * argument or capacity of the problem statement (Secs. 2-3: positions, cell,
 * parameters, cutoff, Krylov order, chemical potential or electron count) was
 * refused, or the HIP runtime's error text. The string is owned by the
 * library and stays valid until the thread's next failing call. Never fails. */
const char *tb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TBKRYLOV_H */
