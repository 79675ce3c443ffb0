// Internal declarations of libmag: context, device buffers, kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <map>
#include <vector>

#include "mag.h"

namespace mag {

constexpr int NORB = MAG_NORB;
constexpr int NU_MAX = MAG_NU_MAX;
constexpr int CLUSTER_MAX = MAG_CLUSTER_MAX;
constexpr int BLOCKS_MAX = MAG_BLOCKS_MAX;
constexpr int PAT_MAX = NORB * BLOCKS_MAX;      // pattern entries of one CSR row
constexpr int NC_MAX = NORB * CLUSTER_MAX;      // cluster orbitals
constexpr double G_SPIN = 2.0;
constexpr int CSLOT_BYTES = 272;  // LDS bytes per cached H/S block (256 + bank pad)

// error flags raised by kernels (bit mask in a device int)
enum KernelError : int {
  KERR_NONE = 0,
  KERR_NOTPD = 1,       // projected overlap not positive definite
  KERR_NONFINITE = 2,   // NaN / Inf met
  KERR_PATTERN = 4,     // a pattern atom outside the cluster
  KERR_CAPACITY = 8,    // a fixed-size buffer would overflow
  KERR_LAYOUT = 16,     // CSR not block-complete
  KERR_BRACKET = 32,    // no sign change of N(mu) - N_e in the bracket
  KERR_NOCONV = 64,     // projected eigensolver hit its iteration limit
};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  uint64_t epoch = 0;  // counts allocations: contents older than it are gone
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  // grow-only allocation; contents are not preserved
  hipError_t reserve(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    release();
    if (n == 0) n = 256;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    bytes = n;
    ++epoch;
    return hipSuccess;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

// state of the chemical-potential search and of the energy sums (device)
struct MuState {
  double lo, hi, mu;
  double E, S_ent, N;
  double ne, kT, tol;
  int done;
  int levels;
  int err;
  unsigned counter;
  double emin, emax;
  double pad[4];
};

struct KrylovArgs {
  const int32_t* bptr;     // N + 1 block-row pointers
  const int32_t* bcol;     // block column atom ids
  const double* bval;      // nblk x 32: H block then S block, each as quarters (columns 0-1, 2-3) of row pairs
  const int64_t* clus_ptr; // N + 1
  const int32_t* clus_atoms;
  const int32_t* cols;     // columns of this launch, in slot order
  int64_t ncols;
  int32_t* queue;          // persistent: one counter per queue, or nullptr (one column per WG)
  const int64_t* qbeg;     // persistent: slot range [qbeg[q], qbeg[q+1]) of queue q
  int nqueue;              // persistent: number of queues (workgroup w starts on queue w % nqueue)
  int nu;                  // requested Krylov dimension (<= template capacity)
  double breakdown;
  double* hs;              // per slot: h (NU x NU, column k rows i<=k) then s
  double* urow;            // per slot: row l of Q (NU)
  double* qpat;            // per slot: pat_stride x cap rows of Q on the pattern
  int32_t* nu_eff;         // per slot
  int32_t* npat;           // per slot: rows written to qpat
  int32_t* err;            // error flag bits
  int cap;                 // NU capacity used for strides
  int pat_stride;          // rows per slot in qpat (PAT_MAX, or NC_MAX when full)
  int full;                // 1: write every cluster row of Q, not only the pattern
  int cache_cap;           // cluster blocks kept in LDS for the whole column (dynamic LDS)
  const int32_t* slots;    // nullptr: list position = slot; else the slots of this launch
  // for the exact gradient (or nullptr): per slot the whole basis (cap columns
  // of adj_rows rows, column k at k * adj_rows), the last step's residual
  // H q_n - Q h[:, n-1] (adj_rows), h (cap x cap, column k rows i <= k) and
  // beta_k (cap)
  double* adj_q;
  double* adj_r;
  double* adj_h;
  double* adj_beta;
  int adj_rows;
};

// how the Krylov columns of one bucket of cluster sizes are launched
struct KrylovPlan {
  int shape = -1;          // workgroup shape (index into the shape table)
  size_t dyn = 0;          // dynamic LDS bytes per workgroup (block cache)
  int cache = 0;           // cached blocks that dyn holds
  int per_cu = 1;          // persistent workgroups per CU
  bool tuned = false;      // timed against the other candidates
  double us_per_col = 0.0; // measured time per column when tuned
  int candidates = 0;      // plans timed (1: nothing to choose)
};

struct KrylovShapeInfo {
  int cap;   // nu capacity (template)
  int tpb;   // threads per workgroup
  int r;     // cluster rows per thread
  const void* unused;
  int id = -1;
  int rows() const { return tpb * r; }
};

struct EigArgs {
  double* hs;                 // projected pencils; overwritten by the reduction
  const double* urow;
  const double* qpat;
  const int32_t* nu_eff_in;   // per slot
  const int32_t* cols;        // per slot global column
  const int64_t* rowptr;      // CSR row pointers (M + 1)
  int64_t ncols;
  int cap;                    // stride capacity of hs/urow/qpat
  int nu;                     // stride of eps/w outputs
  double* eps;                // M x nu (indexed by global column)
  double* w;                  // M x nu
  int32_t* nu_eff_out;        // M
  const int32_t* npat;        // per slot pattern rows
  double* P;                  // Y d on the pattern, or nullptr
  int pmode;                  // 1: P row base = rowptr[j]; 0: slot * pat_stride
  int pat_stride;
  int out_by_slot;            // 1: eps/w/nu_eff rows indexed by slot instead of column
  int32_t* err;
  // eigensolver scratch, per slot
  double* trid;               // 4 cap: d, e, beta of the tridiagonal; s e_1
  double* evu;                // cap: eigenvalues in QL order
  double* rot;                // 2 rec_cap: recorded plane rotations (sn, cs)
  int32_t* sweep;             // sweep_cap: (ms << 8) | count of each QL sweep
  int32_t* qlst;              // number of sweeps, or < 0: finished by the fallback kernel
  int32_t* fb_list;           // slots for the fallback kernel
  int32_t* fb_count;          // 1
  int rec_cap;
  int sweep_cap;
  // exact gradient (optional): the Ritz vectors c (per slot cap x cap, vector
  // k at k * cap) and (eigenvalue, d, g) of each (per slot 3 x cap), in the
  // solver's own order
  double* cvec;
  double* cdg;
};

struct DensityArgs {
  const double* P;
  int pmode;              // as in EigArgs
  int pat_stride;
  const int32_t* cols;    // per slot
  const int64_t* rowptr;
  const double* eps;
  const int32_t* nu_eff;
  int64_t ncols;
  int nu;
  const MuState* st;
  double* rho;
  double* pi;
};

// --------------------------------------------------------------------------
// launchers (implemented in the .hip files)
// --------------------------------------------------------------------------
hipError_t launch_krylov(const KrylovArgs& a, int shape, size_t dyn_lds, int grid, hipStream_t s);
int krylov_shapes(int cap, KrylovShapeInfo* out, int max_out);  // shapes for a nu capacity
size_t krylov_static_lds(int shape);
int krylov_cache_blocks(size_t dyn_lds);
int krylov_occupancy(int shape, size_t dyn_lds);  // workgroups per CU (0: does not fit)
constexpr int KRYLOV_QUEUES = 8;  // one work queue per XCD
int krylov_capacity(int nu);  // template capacity used for nu (0 if unsupported)
hipError_t launch_eig(const EigArgs& a, hipStream_t s);
int eig_rec_cap(int cap);
int eig_sweep_cap(int cap);
hipError_t launch_density(const DensityArgs& a, hipStream_t s);


hipError_t launch_mu_setup(MuState* st, double ne, double kT, double tol, double mu_fixed,
                           int fixed, hipStream_t s);
hipError_t launch_mu_init(const double* eps, const double* w, const int32_t* nu_eff, int64_t M,
                          int nu, MuState* st, double* partials, int grid, hipStream_t s);
hipError_t launch_mu_round(const double* eps, const double* w, const int32_t* nu_eff, int64_t M,
                           int nu, MuState* st, double* partials, int grid, hipStream_t s);
hipError_t launch_energy(const double* eps, const double* w, const int32_t* nu_eff, int64_t M,
                         int nu, MuState* st, double* partials, int grid, hipStream_t s);
int mu_points_per_round();
int mu_levels_per_round();

// clusters
hipError_t launch_cluster_scan_cv(const double* pos, int64_t n, const double cell[3], double rc,
                                  const struct CellList& cl, int32_t* tmp, int32_t* cnt,
                                  int32_t* err, hipStream_t s);
hipError_t launch_cluster_nnz(const int32_t* bptr, const int32_t* bcol, const int64_t* clus_ptr,
                              const int32_t* clus_atoms, int64_t n, int64_t* out, hipStream_t s);
hipError_t launch_cluster_compact(const int32_t* tmp, const int32_t* cnt, const int64_t* ptr,
                                  int64_t n, int32_t* atoms, hipStream_t s);

// cell list (shared by the SK pattern and the clusters)
struct CellList {
  int ncell[3] = {0, 0, 0};
  bool brute = true;
  DevBuf cell_of, cell_count, cell_start, cell_atoms;
};
hipError_t build_cell_list(CellList& cl, const double* pos_dev, int64_t n, const double cell[3],
                           double rmin, hipStream_t s);

// Slater-Koster
struct SKModelDev {
  double es, ep;
  double vh[4];  // ss, sp, pp_sigma, pp_pi for H
  double vs[4];  // same for S - I
  double r0, r_on, r_cut;
};
// exact gradient of the truncated-Krylov grand potential (adjoint.hip)
// basis columns staged per pass of the exact gradient's contraction: each
// pass evaluates the pair derivatives of every cluster block once, so wider
// passes evaluate them fewer times (ten: three passes at nu = 30, whose
// kernel then holds 163,296 of the 163,840 bytes of LDS of a CU)
constexpr int ADJ_KC = 10;
struct AdjointArgs {
  const int32_t* bptr;
  const int32_t* bcol;
  const double* bval;
  const int64_t* clus_ptr;
  const int32_t* clus_atoms;
  const double* pos;       // N x 3
  double box[3];
  SKModelDev m;
  const int32_t* cols;     // columns of the chunk in slot order, the four of an atom together
  int64_t natoms;          // atoms of the chunk (slots 4 a .. 4 a + 3)
  int nu;
  double breakdown;
  const double* hbar;      // per slot: hbar (cap x cap) then sbar
  const int32_t* nu_eff;   // per slot, from the first pass over the chunk
  double* wbar;            // per workgroup: nu x (rows) scratch
  double* fJ;              // per atom J: its parts for its cluster atoms, at 3 clus_ptr[J]
  int32_t* counter;        // atom counter of the persistent workgroups
  int32_t* err;
  int cap;
  // the forward pass's basis, last residual, h and beta per slot (layouts as
  // the Krylov kernel's adj_* outputs)
  const double* q;
  const double* r;
  const double* h;
  const double* beta;
  int qrows;
};
int adjoint_supported(int cap);
size_t adjoint_dyn_lds(int cap);
size_t adjoint_scratch_per_wg(int cap);
int adjoint_occupancy(int cap);
hipError_t launch_adjoint(const AdjointArgs& a, int grid, hipStream_t s);
hipError_t launch_adj_prep(const double* cvec, const double* cdg, const int32_t* nu_eff,
                           int64_t ncols, int cap, const MuState* st, double* hbar, hipStream_t s);
hipError_t launch_gather_forces(const int64_t* clus_ptr, const int32_t* clus_atoms, int64_t n,
                                const double* fJ, double* F, hipStream_t s);


hipError_t launch_sk_count(const double* pos, int64_t n, const double cell[3], double rc,
                           const CellList& cl, int32_t* cnt, int32_t* err, hipStream_t s);
hipError_t launch_sk_fill(const double* pos, int64_t n, const double cell[3], double rc,
                          const CellList& cl, const int32_t* bptr, int32_t* bcol, hipStream_t s);
hipError_t launch_sk_csr(const int32_t* bptr, const int32_t* bcol, int64_t n, int64_t* rowptr,
                         int32_t* colind, hipStream_t s);
hipError_t launch_sk_values(const SKModelDev& m, const double* pos, int64_t n,
                            const double cell[3], const int32_t* bptr, const int32_t* bcol,
                            double* H, double* S, hipStream_t s);
hipError_t launch_icohp(const SKModelDev& m, const double* pos, int64_t n, int64_t nblk,
                        const double cell[3], const int32_t* bptr, const int32_t* bcol,
                        const double* bval, const double* rho, double* B, double* Bsig,
                        double* Bpi, hipStream_t s);
hipError_t launch_pair_rep(const SKModelDev& m, const double* pos, int64_t n, const double cell[3],
                           const int32_t* bptr, const int32_t* bcol, double phi0, double mexp,
                           double* e, double* F, hipStream_t s);
// COCG Green's-function columns (cocg.hip): energies per launch
constexpr int COCG_NZ = 4;
struct CocgArgs {
  const int32_t* cols;  // global column ids
  int64_t ncols;
  const int64_t* clus_ptr;
  const int32_t* clus_atoms;
  const int32_t* bptr;
  const int32_t* bcol;
  const double* bval;  // block values, H then S per 4x4 block
  const double* z;     // all energies (re, im)
  int nz;              // number of energies
  int q0;              // first energy of this launch
  double tol;          // |r| <= tol (|b| = 1)
  int max_iter;
  const int64_t* off;  // output row offsets per column (n + 1)
  double* G;           // complex out, G[2 (off[i] nz + q len_i + c)]
  int32_t* iters;      // per column and energy: steps, or -1
  int32_t* err;
};
hipError_t launch_cocg(const CocgArgs& a, hipStream_t s);
// MD step helpers (md.hip)
hipError_t launch_md_kick(double* v, const double* F, int64_t n3, double c, hipStream_t s);
hipError_t launch_md_drift(double* x, const double* v, int64_t n, double dt, const double cell[3],
                           hipStream_t s);
hipError_t launch_axpy(double* y, const double* x, int64_t n, double a, hipStream_t s);
hipError_t launch_sum(const double* a, int64_t n, int squares, double* out, hipStream_t s);
extern const double AMU_A2_FS2_EV;
// allocation-free entry point (noalloc.hip): the fixed per-device scratch
constexpr int64_t NOALLOC_MAX_BLOCKS = MAG_NOALLOC_MAX_BLOCKS;
constexpr size_t NOALLOC_DOUBLES = (size_t)3 * NOALLOC_MAX_BLOCKS + NOALLOC_MAX_BLOCKS / 2;
void noalloc_init(int device);                      // once per device, that device current
hipError_t noalloc_scratch(int device, void** ptr);  // its device address
hipError_t launch_sk_vjp(const SKModelDev& m, const double* pos, int64_t n, int64_t nblk,
                         const double cell[3], const int32_t* bptr, const int32_t* bcol,
                         const int32_t* btrans, const double* gH, const double* gS, double sign_gS,
                         double* part, double* grad, hipStream_t s);

// system conversion
hipError_t launch_check_layout(const int64_t* rowptr, const int32_t* colind, int64_t n,
                               const int32_t* bptr, int32_t* bcol, int32_t* err, hipStream_t s);
hipError_t launch_to_blocks(const int64_t* rowptr, const double* H, const double* S, int64_t n,
                            const int32_t* bptr, double* bval, hipStream_t s);
hipError_t launch_block_transpose(const int32_t* bptr, const int32_t* bcol, int64_t n,
                                  int32_t* btrans, int32_t* err, hipStream_t s);
hipError_t launch_check_finite(const double* x, int64_t n, int32_t* err, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s);
hipError_t launch_scale_copy(const double* x, int64_t n, double a, double* y, hipStream_t s);
hipError_t launch_cluster_rho(const double* P, int pat_stride, const int32_t* cols, int64_t ncols,
                              const int32_t* npat, const int64_t* out_off, const double* eps,
                              const int32_t* nu_eff, int nu, const MuState* st, double* out,
                              hipStream_t s);
hipError_t launch_cohp(const double* bval, const int32_t* bptr, int64_t n, int64_t nblk,
                       const int64_t* rowptr, const double* P, const double* eps,
                       const int32_t* nu_eff, int nu, const double* en, int ne, double eta,
                       double* out, hipStream_t s);
hipError_t launch_green(const double* P, int pat_stride, const int32_t* cols, int64_t ncols,
                        const int32_t* npat, const int64_t* out_off, const double* eps,
                        const int32_t* nu_eff, int nu, const double* z, int nz, double* out,
                        hipStream_t s);

}  // namespace mag

// the opaque context of the C ABI
struct mag_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;

  // Slater-Koster build
  bool sk_built = false;
  int64_t sk_n = 0, sk_nnz = 0, sk_nblk = 0;
  double sk_cell[3] = {0, 0, 0};
  mag::SKModelDev sk_model{};
  mag::DevBuf sk_pos, sk_bptr, sk_bcol, sk_rowptr, sk_colind, sk_H, sk_S;
  mag::DevBuf md_x, md_v, md_F, md_Frep, md_e, md_sum;  // MD step state
  mag::DevBuf f_part, f_grad;  // force contraction: per-block parts, per-atom sums
  mag::DevBuf adj_cvec, adj_cdg, adj_hbar, adj_wbar, adj_fJ, adj_F, adj_counter;  // exact gradient
  mag::DevBuf adj_q, adj_r, adj_h, adj_beta;  // the forward pass's Krylov data for it
  mag::DevBuf adj_nu;  // the kept pass's column dimensions
  bool adj_kept = false;  // the last solve kept every column's exact-gradient inputs
  // set-up scratch kept between calls (an MD frame rebuilds pattern and clusters)
  mag::CellList sk_cells, sys_cells;
  mag::DevBuf sk_cnt, sys_tmp, sys_cnt, sys_nz;

  // system
  bool has_system = false;
  int64_t N = 0, M = 0, nnz = 0, nblk = 0;
  double cell[3] = {0, 0, 0};
  double r_cluster = 0.0;
  bool has_pos = false;
  mag::DevBuf rowptr, bptr, bcol, btrans, bval, pos, clus_ptr, clus_atoms;
  int64_t clus_total = 0;
  std::vector<int32_t> h_clus_size;   // atoms per cluster
  std::vector<int32_t> h_bcount;      // blocks per block row
  std::vector<int64_t> h_rowptr;      // CSR row pointers (host copy)
  std::vector<int32_t> h_order;       // columns in spatial (Morton) order of their atoms
  std::vector<int64_t> h_qbeg;        // slot ranges of the per-XCD queues over h_order
  int64_t sum_cluster_nnz = 0;

  // solve state
  bool solved = false;
  bool density_ready = false;
  mag_opts opts{};
  int nu = 0;
  mag::DevBuf eps, w, nu_eff, state, partials, P, rho, pi;
  mag::DevBuf k_hs, k_urow, k_qpat, k_nu, k_npat, k_cols, k_queue, k_qbeg, errflag;
  mag::DevBuf k_trid, k_evu, k_rot, k_sweep, k_qlst, k_fbl, k_fbc, k_slots;
  // Krylov launch plan per (nu capacity, workgroup shape of the bucket)
  std::map<std::pair<int, int>, mag::KrylovPlan> kplans;
  // generations: bumped when a device buffer moves / the system changes
  uint64_t alloc_gen = 0, sys_gen = 0;
  // captured forward solve (schedule MAG_SCHED_GRAPH)
  struct Graph {
    hipGraphExec_t exec = nullptr;
    uint64_t alloc_gen = 0, sys_gen = 0;
    mag_opts key{};
    int rounds = 0;
    mag::DevBuf slots, qbeg, queue;  // column lists of the captured launches
  } graph;
  mag::MuState* h_state_pinned = nullptr;  // read back at the end of a captured solve
  hipStream_t aux_stream = nullptr;        // capture stream when the context's is the null stream
  mag::DevBuf tmp_cols, tmp_off, tmp_out;
  int64_t batch_cols = 0;
  mag::MuState h_state{};

  mag_stats stats{};
  // per-launch timing events of the Krylov and eigensolver kernels (pass 1),
  // read after the solve's one synchronisation
  std::vector<hipEvent_t> ev_pool;
  bool time_kernels = false;
  size_t timed_launches = 0;
  // stage timing events (start, end pairs), read after a synchronisation
  std::vector<hipEvent_t> ev_span;
  // pinned host memory that results are copied into in stream order, so
  // that a call reads them after its one synchronisation: words 0-7 the
  // kernel error flags, words 8-15 up to four doubles
  int32_t* h_flags = nullptr;
  bool pass2_pending = false;  // pass 2 enqueued, its flags not checked yet
  // the launch lists of the last single-chunk pass over h_order, resident in
  // k_slots and k_qbeg (valid while the system, nu capacity and buffers stay)
  struct OrderLists {
    bool valid = false;
    uint64_t sys_gen = 0;
    int cap = 0;
    uint64_t slots_epoch = 0, qbeg_epoch = 0;
    std::vector<int8_t> bucket;
    std::vector<int32_t> hslots;
    std::vector<int64_t> hqbeg, boff;
  } lists;
};
