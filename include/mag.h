/*
 * mag.h -- multiple-Arnoldi Green's-function engine for MI355X (gfx950).
 *
 * C ABI of libmag.so.  The library computes, column by column, the Green's
 * function G = (zS - H)^-1 of a sparse real-symmetric tight-binding pencil
 * (H, S), S positive definite, in the LCAO basis (the generalized shifted
 * linear equation, Eq. 1 of arXiv:1210.1531), by one Krylov subspace per
 * column j over the local cluster of j's atom ("multiple Arnoldi" method,
 * parallel over j).  From the Ritz data it forms the Fermi-Dirac density
 * matrix rho (Eq. 2), the chemical potential mu by bisection between the two
 * Green's-function passes of the memory-saving workflow (Eq. 3), the band and
 * free energy, their derivatives dA/dH = rho and dA/dS = -pi (pi = energy
 * density matrix) and, through Slater-Koster derivatives, atomic forces.
 *
 * Conventions shared by every entry point
 *   - Status: MAG_OK (0) or a negative mag_status; mag_last_error() returns a
 *     message for the last failing call on that context.  No C++ exception
 *     crosses the ABI.  Output buffers are unspecified after an error.
 *   - mem_kind: MAG_HOST means the caller's pointers are host memory,
 *     MAG_DEVICE means device memory on the context's device.  Inputs are
 *     copied during the call (they need to stay valid only until it returns);
 *     outputs go to caller-allocated buffers of the documented size.
 *   - Work is queued on the context's stream; every entry point returns after
 *     its outputs (device or host) are complete.
 *   - One context is not thread-safe; distinct contexts are independent.
 *   - Units: energies eV, lengths Angstrom, forces eV/Angstrom.
 *   - Basis: every atom carries MAG_NORB = 4 orbitals (s, px, py, pz); basis
 *     index i = 4 I + alpha for atom I and orbital alpha (the (I, alpha)
 *     decomposition of the COHP paragraph); M = 4 N.
 *   - CSR layout of H, S, rho, pi ("block-complete"): row r = (J, alpha)
 *     lists, for every atom K of the block row of J in ascending order, the
 *     four columns 4K .. 4K+3; the block rows of the four rows of an atom are
 *     identical and include J itself.  Entry p of row r, column c of the
 *     density outputs holds rho_{c r} as obtained from column r, i.e. the
 *     coefficient of H_{r c} in E_band = sum_r sum_c H_{r c} rho_{c r}.
 *   - Environment, read when a context first needs the value:
 *     MAG_SCRATCH_GB (default 8) bounds the per-column scratch of one chunk
 *     of columns; MAG_AUTOTUNE=0 keeps every Krylov launch plan at its
 *     default instead of timing the candidates; MAG_LDS_CACHE=0 makes new
 *     plans stream every matrix block instead of caching a cluster's first
 *     blocks in LDS.  At nu <= 30 the last two change no result bit.
 */
#ifndef MAG_H
#define MAG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MAG_NORB 4
#define MAG_NU_MAX 48       /* largest Krylov dimension */
#define MAG_CLUSTER_MAX 192 /* largest cluster, atoms (768 orbitals) */
#define MAG_BLOCKS_MAX 32   /* largest block row (atoms within r_cut, self included) */
#define MAG_STATS_BUCKETS 8 /* launch plans reported per pass (cluster-size buckets) */

typedef struct mag_ctx mag_ctx;

enum mag_status {
  MAG_OK = 0,
  MAG_EINVAL = -1,      /* bad argument, size or layout */
  MAG_ENOMEM = -2,      /* device allocation failed */
  MAG_EHIP = -3,        /* HIP runtime error */
  MAG_ENOTPD = -4,      /* a projected overlap s = V^T S V is not positive definite */
  MAG_EBRACKET = -5,    /* n_electrons outside (0, 2M) or no sign change in the bracket */
  MAG_ESTATE = -6,      /* call out of order (e.g. density before solve) */
  MAG_ENONFINITE = -7,  /* NaN or Inf in the input or in an intermediate result */
  MAG_EUNSUPPORTED = -8, /* size beyond a documented limit */
  MAG_ENOCONV = -9       /* the projected eigensolver did not converge */
};

enum mag_mem { MAG_HOST = 0, MAG_DEVICE = 1 };

/* Memory workflow of Eq. 3.  RECOMPUTE: pass 1 keeps only the spectral data
 * (eps, w) needed for mu and recomputes every Krylov column for rho in pass 2
 * (the letter's memory-saving workflow).  STORE: pass 1 also keeps Y d on the
 * pattern (n_pat x nu doubles per column) and pass 2 reads it back.  AUTO:
 * STORE when that buffer (nnz x nu doubles) takes at most half of the free
 * device memory (counting a buffer the context already holds for it),
 * RECOMPUTE otherwise. */
enum mag_workflow {
  MAG_WORKFLOW_RECOMPUTE = 0,
  MAG_WORKFLOW_STORE = 1,
  MAG_WORKFLOW_AUTO = 2
};

/* Launch schedule of the per-column Krylov kernels.  Columns are grouped into
 * buckets by cluster size; each bucket runs in the workgroup shape and
 * occupancy that the library timed fastest on first use.  PERSISTENT: per
 * bucket, one launch of resident workgroups pulling columns from eight
 * device queues of spatially contiguous columns (one per XCD, with
 * stealing).  GRID: per bucket, one launch with one workgroup per column.
 * PLAIN: one launch per column.  GRAPH: PERSISTENT launches, with the whole
 * forward solve (Krylov passes, eigensolves, bisection for mu, energies)
 * captured once in a HIP graph and replayed by later solves with the same
 * system and options; the first call runs eagerly, and a graph is captured
 * again whenever a device buffer it uses has moved.  AUTO: PERSISTENT.
 * Per-column results are bitwise identical across schedules. */
enum mag_schedule {
  MAG_SCHED_AUTO = 0,
  MAG_SCHED_PERSISTENT = 1,
  MAG_SCHED_GRID = 2,
  MAG_SCHED_PLAIN = 3,
  MAG_SCHED_GRAPH = 4
};

/* ---------------------------------------------------------------------- */
/* context                                                                  */
/* ---------------------------------------------------------------------- */

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t to
 * enqueue on, or NULL to let the context create its own (default priority).
 * Errors: MAG_EINVAL (out == NULL, bad device), MAG_EHIP. */
int mag_create(mag_ctx** out, int device, void* hip_stream);

/* Free every device buffer of the context (no-op on NULL). */
void mag_destroy(mag_ctx* ctx);

/* Message of the last failing call on ctx ("" if none); valid until the next
 * call on ctx.  Never NULL. */
const char* mag_last_error(const mag_ctx* ctx);

/* ABI version (major * 10000 + minor * 100 + patch). */
int mag_version(void);

/* ---------------------------------------------------------------------- */
/* A0: Slater-Koster two-center sp model (the tight-binding form of H, S)   */
/* ---------------------------------------------------------------------- */

/* Two-center model.  For atoms I, K with d = R_K - R_I, r = |d|, direction
 * cosines l = d / r and radial factor u(r) = (r0/r)^2 fc(r),
 * fc = 1 - (10 t^3 - 15 t^4 + 6 t^5), t = clip((r - r_on)/(r_cut - r_on)):
 *   block_ss = V_ss u, block_s,a = l_a V_sp u, block_a,s = -l_a V_sp u,
 *   block_a,b = (l_a l_b V_pps + (delta_ab - l_a l_b) V_ppp) u
 * with (V_ss, V_sp, V_pps, V_ppp) = the v_* fields for H and the s_* fields
 * for S - I.  Onsite: H = diag(es, ep, ep, ep), S = I.  Pattern: atom pairs
 * closer than r_cut (minimum image in the orthorhombic box) plus each atom
 * with itself.  Requires 2 r_cut < every box length. */
typedef struct {
  double es, ep;
  double v_ss_sigma, v_sp_sigma, v_pp_sigma, v_pp_pi;
  double s_ss_sigma, s_sp_sigma, s_pp_sigma, s_pp_pi;
  double r0, r_on, r_cut;
} mag_sk_model;

/* Build pattern and values of H and S from positions on the device.
 * pos: n_atoms x 3 doubles (mem_kind); cell: 3 box lengths (host).
 * On success *nnz_out = number of CSR nonzeros; fetch the CSR with
 * mag_sk_get_csr.  Errors: MAG_EINVAL (sizes, 2 r_cut >= box),
 * MAG_EUNSUPPORTED (more than MAG_BLOCKS_MAX atoms in a block row),
 * MAG_ENONFINITE, MAG_ENOMEM. */
int mag_sk_build(mag_ctx* ctx, const mag_sk_model* model, int64_t n_atoms,
                 const double* pos, const double cell[3], int mem_kind,
                 int64_t* nnz_out);

/* Copy the CSR built by the last mag_sk_build: rowptr (M+1), colind (nnz),
 * H (nnz), S (nnz).  Any pointer may be NULL to skip it.  MAG_ESTATE if no
 * build was done. */
int mag_sk_get_csr(mag_ctx* ctx, int64_t* rowptr, int32_t* colind, double* H,
                   double* S, int mem_kind);

/* Recompute H and S values on the pattern of the last build for new
 * positions pos (n_atoms x 3); the pattern is kept even if atoms cross
 * r_cut (the smooth cutoff makes such entries vanish there). */
int mag_sk_values(mag_ctx* ctx, const double* pos, double* H, double* S,
                  int mem_kind);

/* Vector-Jacobian product of the SK map on the built pattern:
 * grad[I] = sum_p gH[p] dH_p/dR_I + gS[p] dS_p/dR_I  (n_atoms x 3). */
int mag_sk_vjp(mag_ctx* ctx, const double* pos, const double* gH,
               const double* gS, double* grad, int mem_kind);

/* Allocation-free variant of mag_sk_vjp, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops and
 * harnesses that forbid hipMalloc.  The same product on the pattern of the
 * last mag_sk_build, grad[I] = sum_p gH[p] dH_p/dR_I + gS[p] dS_p/dR_I, with
 * the same kernels and results bitwise equal to mag_sk_vjp's; its
 * intermediates (the per-block parts and the block transposes) live in a
 * fixed per-GPU array of MAG_NOALLOC_MAX_BLOCKS x 28 bytes (28 MiB) that
 * each GPU the library runs on holds until the process ends, and the call
 * allocates and frees nothing.  pos (n_atoms x 3), gH, gS (nnz each) and
 * grad (n_atoms x 3) are device memory on the context's device (checked;
 * host pointers are rejected).  The context's positions are left as they
 * are.  Every call on one GPU uses that GPU's one array, so calls that
 * overlap on a GPU (other threads or contexts on other streams) race.
 * Errors: MAG_ESTATE without a build, MAG_EINVAL (NULL or non-device
 * pointers, a pattern without transposed blocks), MAG_EUNSUPPORTED (more than
 * MAG_NOALLOC_MAX_BLOCKS blocks in the pattern), MAG_EHIP. */
#define MAG_NOALLOC_MAX_BLOCKS 1048576
int mag_sk_vjp_noalloc(mag_ctx* ctx, const double* pos, const double* gH, const double* gS,
                       double* grad);

/* ---------------------------------------------------------------------- */
/* system (H, S, clusters)                                                  */
/* ---------------------------------------------------------------------- */

typedef struct {
  int64_t n_atoms;           /* N */
  int64_t nnz;               /* CSR nonzeros */
  const int64_t* rowptr;     /* M + 1, block-complete layout (see top) */
  const int32_t* colind;     /* nnz */
  const double* H;           /* nnz, eV */
  const double* S;           /* nnz */
  const double* pos;         /* N x 3, needed when clusters are built here and for forces */
  double cell[3];            /* orthorhombic box lengths */
  double r_cluster;          /* cluster radius; <= 0, or 2 r >= min box length: whole cell */
  const int64_t* clus_ptr;   /* N + 1, or NULL to build clusters from pos */
  const int32_t* clus_atoms; /* ascending atom ids of each cluster, or NULL */
} mag_system;

/* Set the pencil and the clusters.  The cluster of atom J (a reading of the
 * letter's column-parallel generation of G) holds every atom I with
 * |R_I - R_J| <= r_cluster (minimum image, inclusive), J included, with all
 * four orbitals, ordered by atom id then orbital.  Every atom of J's block row
 * must lie in J's cluster.  Errors: MAG_EINVAL (layout not block-complete,
 * sizes), MAG_EUNSUPPORTED (cluster larger than MAG_CLUSTER_MAX atoms),
 * MAG_ENONFINITE, MAG_ENOMEM. */
int mag_set_system(mag_ctx* ctx, const mag_system* sys, int mem_kind);

/* Replace the values of H and S (same pattern, nnz each). */
int mag_update_values(mag_ctx* ctx, const double* H, const double* S, int mem_kind);

/* Copy the clusters in use: clus_ptr (N+1) and clus_atoms (clus_ptr[N]).
 * Either pointer may be NULL; *total_out (may be NULL) receives clus_ptr[N]. */
int mag_get_clusters(mag_ctx* ctx, int64_t* clus_ptr, int32_t* clus_atoms,
                     int64_t* total_out, int mem_kind);

/* ---------------------------------------------------------------------- */
/* forward: Krylov columns, mu, energy                                      */
/* ---------------------------------------------------------------------- */

typedef struct {
  int nu;             /* Krylov dimension, 1 .. MAG_NU_MAX (clamped per column to 4|C|) */
  double kT;          /* Fermi-Dirac temperature, eV, > 0 */
  double n_electrons; /* electron count, 0 < n_electrons < 2 M (spin factor 2) */
  double mu_tol;      /* bisection stops when the bracket is <= mu_tol (<= 0: 1e-12 eV) */
  double mu_fixed;    /* NaN: find mu by bisection; else use this mu */
  double breakdown;   /* Krylov breakdown threshold, relative (<= 0: 1e-12) */
  int workflow;       /* mag_workflow */
  int schedule;       /* mag_schedule */
  int eig_sweeps;     /* QL sweeps recorded per column (<= 0: the library's cap, 4 nu up
                         to 128); a column that needs more is finished by the one-wave
                         QL that applies its rotations directly (same results to rounding) */
  int keep_exact;     /* 1: pass 1 keeps each column's Krylov basis, h, beta, last residual
                         and Ritz vectors (about (nu + 1) 768 + 4 nu^2 doubles per column) so
                         that a following mag_forces_exact skips its own pass; kept only
                         when every column fits one chunk (MAG_SCRATCH_GB) and nu <= 30 */
} mag_opts;

/* Fill opts with the defaults (nu 30, kT 0.1, n_electrons 0 (must be set),
 * mu_tol 1e-12, mu_fixed NaN, breakdown 1e-12, workflow AUTO, schedule AUTO,
 * eig_sweeps 0, keep_exact 0). */
void mag_opts_default(mag_opts* opts);

/* Pass 1 of Eq. 3 over every column, then mu, then the energies.
 * Per column j = (J, alpha), with l the local index of j in J's cluster C:
 * the Krylov space K_nu(H_C; e_l) (grown by SpMV and re-orthogonalized
 * Gram-Schmidt; the basis is Euclidean-orthonormal, which spans the same
 * space as the S-orthonormal basis of the reading), the projected pencil
 * (h, s) = (Q^T H_C Q, Q^T S_C Q), its eigenpairs h c = eps s c, and the
 * weights w_k = 2 d_k g_k with d = (Qc)^T e_l, g = (Qc)^T S_C e_l.
 * mu solves N(mu) = sum_jk w_jk f((eps_jk - mu)/kT) = n_electrons by
 * bisection (mid = lo + (hi - lo)/2 on [min eps - 40 kT, max eps + 40 kT]).
 * E_band = sum w f eps, A_free = E_band - kT sum w s(f).  Any output pointer
 * may be NULL.  Errors: MAG_ESTATE (no system), MAG_EINVAL (opts),
 * MAG_EBRACKET, MAG_ENOTPD, MAG_ENONFINITE, MAG_ENOCONV. */
int mag_solve_columns(mag_ctx* ctx, const mag_opts* opts, double* mu,
                      double* E_band, double* A_free);

/* Spectral data of the last solve: eps, w (M x nu, row j = column j, entries
 * k >= nu_eff[j] are 0) and nu_eff (M).  Any pointer may be NULL. */
int mag_spectra(mag_ctx* ctx, double* eps, double* w, int32_t* nu_eff, int mem_kind);

/* Energies of the last solve, taken through the density matrix (the method
 * outline after Eq. 1: energy and force through rho; Eq. 2 on the Ritz
 * spectrum): E_band = sum_jk w_jk f_jk eps_jk (= sum_p H_p rho_p), A_free
 * = E_band - kT S_ent (Mermin free energy), the electron count N = sum w f
 * (= sum_p S_p rho_p, the quantity the bisection of the Eq. 3 workflow fixes)
 * and the entropy sum S_ent = sum w s(f).  Any pointer may be NULL; host
 * scalars.  Errors: MAG_ESTATE before a solve. */
int mag_energy(mag_ctx* ctx, double* E_band, double* A_free, double* N_check,
               double* S_ent);

/* Ritz data of selected columns at the current system and opts (no mu, no
 * state change): eps, w (n x nu), nu_eff (n).  For sampled checks at any
 * size.  cols: n global column ids (mem_kind). */
int mag_column_spectra(mag_ctx* ctx, const mag_opts* opts, const int32_t* cols,
                       int64_t n, double* eps, double* w, int32_t* nu_eff,
                       int mem_kind);

/* ---------------------------------------------------------------------- */
/* pass 2: density matrix, Green's function columns                         */
/* ---------------------------------------------------------------------- */

/* rho and pi = energy-density matrix on the CSR pattern of H (nnz each):
 *   rho_ij = 2 sum_k f_k Y_ik d_k,  pi_ij = 2 sum_k f_k eps_k Y_ik d_k,
 * Y = Q c, for i in the block row of j's atom (Eq. 2 on the Ritz spectrum).
 * Runs pass 2 of the last solve's workflow.  pi may be NULL. */
int mag_density_matrix(mag_ctx* ctx, double* rho_csr, double* pi_csr, int mem_kind);

/* Full cluster columns of rho (Eq. 2 on each column's Ritz spectrum, every
 * row of the cluster instead of the pattern; the columns of G generated one
 * by one in the LCAO basis, the paragraph after Eq. 1) at the last solve's
 * mu: for column cols[i] the values rho_{c j} for every orbital c of its
 * cluster in cluster order are written at rho_out[offsets[i] ..
 * offsets[i+1]), offsets[i+1] - offsets[i] = 4 |C(atom of cols[i])|.
 * offsets (n+1, int64, host) is filled by the call; pass rho_out = NULL to
 * get the offsets only.  The Krylov columns are recomputed.  Errors:
 * MAG_ESTATE before a solve, MAG_EINVAL for column ids outside [0, M). */
int mag_cluster_columns(mag_ctx* ctx, const int32_t* cols, int64_t n,
                        double* rho_out, int64_t* offsets, int mem_kind);

/* Columns of the Green's function G = (zS - H)^-1 of Eq. 1 as the method
 * approximates them: the Galerkin columns on each column's Krylov space,
 * G_{c j}(z) = sum_k Y_ck d_k / (z - eps_k) (no spin factor), at nz complex
 * energies z (re, im pairs, host), for every orbital c of the cluster; output
 * complex (re, im) at G_out[2 (offsets[i] * nz + q * len_i + c)] for column
 * i, energy q, local orbital c, with offsets as in mag_cluster_columns.  The
 * Krylov columns are computed with `opts` (nu, breakdown) at the current
 * system.  Errors: MAG_ESTATE without a system, MAG_EINVAL (columns, nz < 1,
 * non-finite z). */
int mag_green_columns(mag_ctx* ctx, const mag_opts* opts, const int32_t* cols,
                      int64_t n, const double* z, int nz, double* G_out,
                      int64_t* offsets, int mem_kind);

/* ---------------------------------------------------------------------- */
/* derivatives                                                              */
/* ---------------------------------------------------------------------- */

/* Adjoint of A_free in the density-matrix reading of the method (energy and
 * force through rho, after Eq. 1; Eq. 2): dA/dH = gA * rho and dA/dS =
 * -gA * pi on the CSR pattern (nnz each, mem_kind; either may be NULL), the
 * coefficients of H and S in E_band and in the electron count.  Runs pass 2
 * of the last solve's workflow (Eq. 3) if needed.  Errors: MAG_ESTATE before
 * a solve. */
int mag_backward(mag_ctx* ctx, double gA, double* dAdH_csr, double* dAdS_csr,
                 int mem_kind);

/* Forces through the density matrix (the method outline after Eq. 1: energy
 * and force through rho): F_I = -sum_p [rho_p dH_p/dR_I - pi_p dS_p/dR_I]
 * (n_atoms x 3, mem_kind) from the density matrices of the last solve (Eq. 2;
 * pass 2 of Eq. 3 runs if needed) and the SK derivatives of `model` at the
 * system's positions.  The derivative of A_free when every column's Krylov
 * space is exact; mag_forces_exact differentiates the truncated method.
 * Requires mag_system.pos and a pattern in the layout of mag_sk_build.
 * Errors: MAG_ESTATE before a solve, MAG_EINVAL (model, F, no positions). */
int mag_forces(mag_ctx* ctx, const mag_sk_model* model, double* F, int mem_kind);

/* Exact forces of the truncated-Krylov method: F_I = -dOmega/dR_I at the
 * last solve's mu, Omega = sum_j Omega_j, Omega_j = sum_k w_jk omega(eps_jk)
 * with omega(e) = -kT ln(1 + exp(-(e - mu)/kT)) (the grand potential; at
 * fixed electron number its position gradient is that of A_free).  The force
 * through rho and pi (mag_forces; the letter takes energy and force through
 * the density matrix, after Eq. 1) is this derivative only when every
 * column's Krylov space is exact; here each column is differentiated through
 * its Krylov space as well: its Ritz data give dOmega_j/dh and dOmega_j/ds of
 * the projected pencil (divided differences of omega), the Krylov recurrence
 * is run backwards with the basis recomputed (no basis is stored), and the
 * resulting dOmega_j/dH_C, dOmega_j/dS_C are contracted with the Slater-Koster
 * derivatives of `model` on the cluster's pairs.  A column whose Krylov space
 * is invariant before nu is differentiated at its dimension.  F: n_atoms x 3
 * (mem_kind).  Requires a solve, mag_system.pos and the pattern of
 * mag_sk_build; supports nu <= 30.  Errors: MAG_ESTATE before a solve,
 * MAG_EINVAL (model, F, no positions), MAG_EUNSUPPORTED (nu > 30). */
int mag_forces_exact(mag_ctx* ctx, const mag_sk_model* model, double* F, int mem_kind);

/* Integrated crystal orbital Hamiltonian populations (Eqs. 4-8) of the last
 * solve, one value per 4x4 block of the pattern, in block-CSR order (block t
 * of block row J, whose column atom K is the t-th atom of row J's CSR
 * blocks; nnz / 16 values per array):
 *   B[b]       = sum_ab H_{Ja;Kb} rho_{Kb;Ja}  (Eq. 5: the COHP integrated
 *                against f, through rho of Eq. 2; spin factor 2 as in rho),
 *   B_sigma[b] = the same with H replaced by its sigma part,
 *   B_pi[b]    = ... by its pi part (the V_pp_pi term of the p-p sub-block),
 * the split taken from the two-center blocks of `model` at the system's
 * positions; B_sigma = B_pi = 0 on the diagonal blocks.  The sum of B over
 * all blocks is E_band (Eq. 6), and B = B_sigma + B_pi on the off-diagonal
 * blocks when H is the model's (Eq. 8).  Any output may be NULL (not all).
 * Requires mag_system.pos; runs pass 2 if needed.  Errors: MAG_EINVAL for a
 * bad model, no outputs or no positions; MAG_ESTATE before a solve. */
int mag_icohp(mag_ctx* ctx, const mag_sk_model* model, double* B, double* B_sigma,
              double* B_pi, int mem_kind);

/* Energy-resolved crystal orbital Hamiltonian populations (Eq. 4) of the
 * last solve, broadened by eta > 0 (z = e + i eta), at ne energies (host
 * array, eV): for block t of block row J (column atom K),
 *   C[b * ne + q] = -(g_s / pi) sum_ab H_{Ja;Kb} Im G_{Kb;Ja}(e_q + i eta)
 * with G the Galerkin columns on the Ritz spectrum, in block-CSR order as in
 * mag_icohp (nnz / 16 blocks).  Integrated against f(e - mu) it tends to the
 * ICOHP B as eta -> 0 (Eq. 5).  Needs the pattern rows kept by the store
 * workflow: MAG_ESTATE after a solve with MAG_WORKFLOW_RECOMPUTE (or before
 * any solve); MAG_EINVAL for ne <= 0, eta < 1e-100 or non-finite energies. */
int mag_cohp(mag_ctx* ctx, const double* energies, int ne, double eta, double* C, int mem_kind);

/* Green's-function columns by a second solver of Eq. 1: the conjugate
 * orthogonal conjugate gradient method (van der Vorst and Melissen), CG with
 * the bilinear form u^T v for the complex symmetric A = z S - H.  Column
 * cols[i] = (J, alpha) solves (z_q S_C - H_C) x = e_l on the cluster of atom
 * J (the same locality as the multiple Arnoldi columns; the column of
 * (z S - H)^-1 itself for a whole-cell cluster), from x = 0, until
 * |r|_2 <= tol or max_iter steps, for nz energies z (re, im pairs, host;
 * every Im z != 0).  Output layout as mag_green_columns: complex (re, im) at
 * G_out[2 (offsets[i] * nz + q * len_i + c)]; offsets (n+1, int64, host) is
 * filled by the call (G_out = NULL: offsets only).  iters (n x nz, int32,
 * mem_kind; may be NULL) receives the steps taken, or -1 where tol was not
 * reached or the method broke down (<p, A p> = 0 or <r, r> = 0); G_out then
 * holds the last iterate.  Four energies share each pass over the cluster's
 * H and S blocks.  Errors: MAG_EINVAL for bad columns, real or non-finite
 * energies, tol <= 0 or max_iter < 1; MAG_ESTATE without a system. */
int mag_cocg_columns(mag_ctx* ctx, const int32_t* cols, int64_t n, const double* z, int nz,
                     double tol, int max_iter, double* G_out, int64_t* offsets,
                     int32_t* iters, int mem_kind);

/* ---------------------------------------------------------------------- */
/* MD step                                                                  */
/* ---------------------------------------------------------------------- */

/* Pair repulsion of the tight-binding total energy on the pattern of the
 * last mag_sk_build (its positions, box and model):
 *   E_rep = sum over atom pairs {I, K} closer than r_cut of
 *           phi(r) = phi0 (r0 / r)^m_rep fc(r),
 * r0 and the smooth cutoff fc (r_on .. r_cut) being the SK model's.  This is
 * the repulsive part that a tight-binding total energy adds to the band
 * energy (the form of Goodwin, Skinner and Pettifor for (r0/r)^2 hoppings).
 * Outputs: *E_rep (host; may be NULL), e_atom (n_atoms: the half of each of
 * an atom's pairs; may be NULL), F (n_atoms x 3: -dE_rep/dR; may be NULL).
 * Errors: MAG_ESTATE without a build; MAG_EINVAL for non-finite phi0 or
 * m_rep <= 0. */
int mag_pair_repulsion(mag_ctx* ctx, double phi0, double m_rep, double* E_rep, double* e_atom,
                       double* F, int mem_kind);

typedef struct {
  double dt;        /* time step, fs (> 0) */
  double mass;      /* mass of every atom, amu (> 0) */
  double phi0;      /* pair repulsion prefactor, eV (0: band energy only) */
  double m_rep;     /* pair repulsion exponent (> 0 when phi0 != 0) */
  double r_cluster; /* cluster radius of every column, Angstrom (<= 0: the whole cell) */
  int n_steps;      /* MD steps (>= 0) */
  int exact_forces; /* 0: forces through rho and pi (mag_forces); 1: the exact gradient of the
                       truncated method (mag_forces_exact, nu <= 30) */
} mag_md_opts;

/* n_steps of velocity Verlet on the potential energy E_pot = A_free + E_rep,
 * each step being the method's unit of work: H and S rebuilt from the model
 * at the new positions (pattern and clusters included), the columns solved
 * with `opts`, the forces taken through the density matrix (mag_forces) plus
 * the pair term, and
 *   v += dt F / (2 m);  x += dt v (wrapped into [0, L));  F = F(x);  v += dt F / (2 m)
 * in units of Angstrom, fs, eV and amu (1 amu A^2/fs^2 = 103.6427 eV).
 * pos and vel (n_atoms x 3, mem_kind) hold the start on entry and the end on
 * return; F (n_atoms x 3, mem_kind; may be NULL) receives the last forces;
 * thermo (host, (n_steps + 1) x 5) receives per frame, the start first:
 * E_pot, E_kin = sum m |v|^2 / 2, mu, E_band, E_rep (eV).  The context holds
 * the last frame's system and solve afterwards (mag_energy, mag_icohp ...).
 * Errors: as mag_sk_build, mag_set_system and mag_solve_columns, for the
 * frame at which they occur (pos and vel then hold that frame); MAG_EINVAL
 * for bad md options or NULL arrays.  With exact_forces the electronic force
 * is the exact derivative of A_free of the truncated method, so E_pot + E_kin
 * is conserved to the integrator's order; through rho it is conserved only
 * when every Krylov space is exact. */
int mag_md_run(mag_ctx* ctx, const mag_sk_model* model, const mag_opts* opts,
               const mag_md_opts* md, int64_t n_atoms, const double cell[3], double* pos,
               double* vel, double* F, double* thermo, int mem_kind);

/* ---------------------------------------------------------------------- */
/* diagnostics                                                              */
/* ---------------------------------------------------------------------- */

typedef struct {
  double t_set_system_ms;  /* last mag_set_system */
  double t_pass1_ms;       /* last pass 1 (Krylov + projected eigensolve) */
  double t_mu_ms;          /* last bisection + energy */
  double t_pass2_ms;       /* last pass 2 */
  double t_forces_ms;      /* last mag_forces */
  int64_t n_columns;       /* M */
  int64_t max_cluster;     /* largest cluster, orbitals */
  int64_t sum_cluster_nnz; /* sum over atoms of nonzeros of H_C */
  int64_t device_bytes;    /* device memory held by the context */
  int32_t bisect_levels;   /* halvings of the last bisection */
  int32_t schedule_used;   /* mag_schedule actually launched */
  double t_krylov_ms;      /* last pass 1: summed durations of the Krylov kernel launches
                              (HIP events on the context stream; 0 for PLAIN) */
  double t_eig_ms;         /* last pass 1: summed durations of the eigensolver launches */
  int32_t krylov_launches; /* Krylov kernel launches in the last pass 1 */
  int32_t workflow_used;   /* mag_workflow of the last solve (never AUTO) */
  int32_t krylov_buckets;  /* cluster-size buckets (workgroup shapes) of the last pass 1 */
  int32_t krylov_tpb;      /* threads per workgroup of the largest bucket's plan */
  double autotune_ms;      /* time spent timing launch plans (first use of a shape) */
  double t_icohp_ms;       /* last mag_icohp (after pass 2) */
  double t_cohp_ms;        /* last mag_cohp */
  double t_md_step_ms;     /* last mag_md_run: average wall time of one step */
  double t_cocg_ms;        /* last mag_cocg_columns (its kernels) */
  double t_forces_exact_ms; /* last mag_forces_exact */
  int32_t krylov_cache_blocks; /* H/S blocks of each cluster held in LDS by the largest bucket's plan */
  /* the launch plan of each cluster-size bucket of the last pass 1 (bucket b
     holds the clusters between the row capacities of the shapes b-1 and b;
     entries of unused buckets are 0) */
  int32_t plan_threads[MAG_STATS_BUCKETS];    /* threads per workgroup */
  int32_t plan_rows[MAG_STATS_BUCKETS];       /* cluster rows per thread */
  int32_t plan_per_cu[MAG_STATS_BUCKETS];     /* persistent workgroups per CU */
  int32_t plan_cache[MAG_STATS_BUCKETS];      /* cluster blocks cached in LDS */
  int32_t plan_candidates[MAG_STATS_BUCKETS]; /* plans timed for the bucket (0: not tuned) */
  int64_t plan_columns[MAG_STATS_BUCKETS];    /* columns of the bucket */
  double plan_us_per_col[MAG_STATS_BUCKETS];  /* the chosen plan's timed us per column */
} mag_stats;

int mag_get_stats(mag_ctx* ctx, mag_stats* out);

#ifdef __cplusplus
}
#endif

#endif /* MAG_H */
