// Host side of the C ABI declared in include/mag.h: context, system set-up,
// the two Green's-function passes of the memory-saving workflow (Eq. 3), the
// chemical potential, energies, derivatives and forces.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <numeric>

#include "mag_internal.h"

using namespace mag;

namespace {

int fail(mag_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

#define HIPCHK(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(ctx, MAG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));      \
  } while (0)

// grow-only device allocation; a buffer that moves invalidates captured graphs.
// A buffer outgrown by a new system (the pattern of an MD frame gaining a
// few blocks) is replaced with 1/16 headroom, so that the next small growth
// does not free and allocate it again.
#define ALLOC(buf, nbytes)                                                                  \
  do {                                                                                     \
    void* old_p_ = (buf).p;                                                                \
    const size_t want_ = (size_t)(nbytes);                                                  \
    const size_t ask_ = ((buf).p && want_ > (buf).bytes) ? want_ + want_ / 16 : want_;     \
    if ((buf).reserve(ask_) != hipSuccess) {                                               \
      (void)hipGetLastError();                                                             \
      return fail(ctx, MAG_ENOMEM, std::string("device allocation of ") +                 \
                                       std::to_string(ask_) + " bytes failed");            \
    }                                                                                      \
    if ((buf).p != old_p_) ++ctx->alloc_gen;                                               \
  } while (0)

#define TRY(expr)                \
  do {                           \
    int rc_ = (expr);            \
    if (rc_ != MAG_OK) return rc_; \
  } while (0)

hipMemcpyKind kind_in(int mem_kind) {
  return mem_kind == MAG_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
}
hipMemcpyKind kind_out(int mem_kind) {
  return mem_kind == MAG_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
}

int check_mem_kind(mag_ctx* ctx, int mem_kind) {
  if (mem_kind != MAG_HOST && mem_kind != MAG_DEVICE)
    return fail(ctx, MAG_EINVAL, "mem_kind must be MAG_HOST or MAG_DEVICE");
  return MAG_OK;
}

int copy_in(mag_ctx* ctx, DevBuf& dst, const void* src, size_t bytes, int mem_kind) {
  ALLOC(dst, bytes);
  if (bytes) HIPCHK(hipMemcpyAsync(dst.p, src, bytes, kind_in(mem_kind), ctx->stream));
  return MAG_OK;
}

int copy_out(mag_ctx* ctx, void* dst, const void* src, size_t bytes, int mem_kind) {
  if (!dst || !bytes) return MAG_OK;
  HIPCHK(hipMemcpyAsync(dst, src, bytes, kind_out(mem_kind), ctx->stream));
  return MAG_OK;
}

int sync(mag_ctx* ctx) {
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return MAG_OK;
}

// words of ctx->h_flags: the flags after a call's last kernel, after pass 1
// of a solve, after pass 2
constexpr int FLAGS_CALL = 0, FLAGS_PASS1 = 1, FLAGS_PASS2 = 2;

// copy the kernel error flags, in stream order, into a pinned host word
int flags_enqueue(mag_ctx* ctx, int slot) {
  HIPCHK(hipMemcpyAsync(ctx->h_flags + slot, ctx->errflag.p, sizeof(int32_t),
                        hipMemcpyDeviceToHost, ctx->stream));
  return MAG_OK;
}

// map flags read back (after a synchronisation) to a status; a set flag is
// cleared on the device
int flags_status(mag_ctx* ctx, int32_t flags, const char* where) {
  if (!flags) return MAG_OK;
  HIPCHK(hipMemsetAsync(ctx->errflag.p, 0, sizeof(int32_t), ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  std::string w(where);
  if (flags & KERR_NONFINITE) return fail(ctx, MAG_ENONFINITE, w + ": non-finite value");
  if (flags & KERR_NOTPD)
    return fail(ctx, MAG_ENOTPD, w + ": projected overlap not positive definite");
  if (flags & KERR_LAYOUT)
    return fail(ctx, MAG_EINVAL, w + ": CSR pattern is not block-complete and symmetric");
  if (flags & KERR_PATTERN)
    return fail(ctx, MAG_EINVAL, w + ": a block-row atom lies outside the column's cluster");
  if (flags & KERR_CAPACITY)
    return fail(ctx, MAG_EUNSUPPORTED, w + ": a cluster or block row exceeds the library limits");
  if (flags & KERR_NOCONV)
    return fail(ctx, MAG_ENOCONV, w + ": the projected eigensolver did not converge");
  return fail(ctx, MAG_EHIP, w + ": kernel error flag " + std::to_string(flags));
}

// read and clear the kernel error flags; map them to a status
int take_errors(mag_ctx* ctx, const char* where) {
  TRY(flags_enqueue(ctx, FLAGS_CALL));
  TRY(sync(ctx));
  return flags_status(ctx, ctx->h_flags[FLAGS_CALL], where);
}

SKModelDev to_dev(const mag_sk_model& m) {
  SKModelDev d;
  d.es = m.es;
  d.ep = m.ep;
  d.vh[0] = m.v_ss_sigma;
  d.vh[1] = m.v_sp_sigma;
  d.vh[2] = m.v_pp_sigma;
  d.vh[3] = m.v_pp_pi;
  d.vs[0] = m.s_ss_sigma;
  d.vs[1] = m.s_sp_sigma;
  d.vs[2] = m.s_pp_sigma;
  d.vs[3] = m.s_pp_pi;
  d.r0 = m.r0;
  d.r_on = m.r_on;
  d.r_cut = m.r_cut;
  return d;
}

bool model_ok(const mag_sk_model* m) {
  if (!m) return false;
  const double v[] = {m->es, m->ep, m->v_ss_sigma, m->v_sp_sigma, m->v_pp_sigma, m->v_pp_pi,
                      m->s_ss_sigma, m->s_sp_sigma, m->s_pp_sigma, m->s_pp_pi, m->r0, m->r_on,
                      m->r_cut};
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return m->r0 > 0.0 && m->r_on > 0.0 && m->r_cut > m->r_on;
}

int device_count_cus(int device) {
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return 256;
  return n > 0 ? n : 256;
}

bool whole_cell(const double cell[3], double rc) {
  const double lmin = std::min(cell[0], std::min(cell[1], cell[2]));
  return rc <= 0.0 || 2.0 * rc >= lmin;
}

// events from a per-context pool (created once, destroyed with the context)
hipEvent_t pool_event(mag_ctx* ctx, size_t i) {
  while (ctx->ev_pool.size() <= i) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ctx->ev_pool.push_back(e);
  }
  return ctx->ev_pool[i];
}

// stage timing without a synchronisation of its own: a start and an end
// event per stage, recorded in stream order and read after the call's
// synchronisation
enum { SPAN_PASS1 = 0, SPAN_MU, SPAN_PASS2, SPAN_FORCES, SPAN_EXACT, SPAN_COUNT };

int span_mark(mag_ctx* ctx, int span, int end) {
  while (ctx->ev_span.size() < 2 * (size_t)SPAN_COUNT) {
    hipEvent_t e = nullptr;
    HIPCHK(hipEventCreate(&e));
    ctx->ev_span.push_back(e);
  }
  HIPCHK(hipEventRecord(ctx->ev_span[2 * span + end], ctx->stream));
  return MAG_OK;
}

double span_ms(mag_ctx* ctx, int span) {
  float ms = 0.f;
  if (ctx->ev_span.size() < 2 * (size_t)SPAN_COUNT ||
      hipEventElapsedTime(&ms, ctx->ev_span[2 * span], ctx->ev_span[2 * span + 1]) !=
          hipSuccess) {
    (void)hipGetLastError();
    return 0.0;
  }
  return ms;
}

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t s;
  explicit Timer(hipStream_t st) : s(st) {
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    (void)hipEventRecord(a, s);
  }
  double stop_ms() {
    float ms = 0.f;
    (void)hipEventRecord(b, s);
    (void)hipEventSynchronize(b);
    (void)hipEventElapsedTime(&ms, a, b);
    return ms;
  }
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// ---------------------------------------------------------------------------
// running the per-column kernels over a list of columns
// ---------------------------------------------------------------------------
struct ColumnJob {
  const int32_t* cols_dev = nullptr;  // device column list (slot order)
  std::vector<int32_t> cols_host;     // same, host copy
  bool order = false;                 // the columns are ctx->h_order (every column)
  int nu = 30;
  double breakdown = 1e-12;
  int eig_sweeps = 0;      // > 0: fewer recorded QL sweeps than the buffers hold
  int keep_adj = 0;        // pass 1 of a solve that keeps the exact gradient's inputs
  int schedule = MAG_SCHED_AUTO;
  int full = 0;            // write every cluster row of Q
  // eig outputs
  double* eps = nullptr;   // spectra rows (by column id or by slot)
  double* w = nullptr;
  int32_t* nu_eff = nullptr;
  int out_by_slot = 0;
  // P and what to do with it
  int want_P = 0;          // compute P = Y d on the rows
  double* P_store = nullptr;  // if set: P goes to this array with base rowptr[j] (pmode 1)
  // per-chunk consumer after the eig kernel
  int consumer = 0;        // 0 none, 1 density on pattern, 2 cluster rho, 3 Green's columns
  double* rho = nullptr;
  double* pi = nullptr;
  const int64_t* out_off = nullptr;  // consumers 2, 3: output offsets by slot (device)
  double* out = nullptr;
  const double* z = nullptr;         // consumer 3: complex energies (device)
  int nz = 0;
  // consumer 4: exact gradient (the chunk's Ritz vectors -> hbar, sbar ->
  // the adjoint sweep and contraction -> per-atom force parts in adj_fJ)
  SKModelDev skm{};
};

// split slots [0, n) of a column list into KRYLOV_QUEUES contiguous ranges of
// about equal work (cluster size as the cost of a column)
std::vector<int64_t> queue_ranges(const mag_ctx* ctx, const int32_t* cols, int64_t n) {
  std::vector<int64_t> beg(KRYLOV_QUEUES + 1, n);
  double total = 0.0;
  for (int64_t i = 0; i < n; ++i) total += ctx->h_clus_size[cols[i] >> 2];
  double acc = 0.0;
  int q = 1;
  beg[0] = 0;
  for (int64_t i = 0; i < n && q < KRYLOV_QUEUES; ++i) {
    acc += ctx->h_clus_size[cols[i] >> 2];
    // cut after whole atoms only (the four columns of an atom stay together)
    const bool atom_end = (i + 1 == n) || ((cols[i + 1] >> 2) != (cols[i] >> 2));
    if (atom_end && acc >= total * q / KRYLOV_QUEUES) beg[q++] = i + 1;
  }
  for (; q <= KRYLOV_QUEUES; ++q) beg[q] = n;
  return beg;
}

// columns per chunk: the per-column scratch of a chunk stays within
// MAG_SCRATCH_GB (default 8 GB)
int64_t chunk_columns(const ColumnJob& job, int64_t n) {
  const int cap = krylov_capacity(job.nu);
  const int pat_stride = job.full ? NC_MAX : PAT_MAX;
  const int rec_cap = eig_rec_cap(cap), sweep_cap = eig_sweep_cap(cap);
  const size_t per_slot =
      sizeof(double) * ((size_t)2 * cap * cap + cap + (size_t)pat_stride * cap) + 2 * sizeof(int32_t) +
      sizeof(double) * ((size_t)5 * cap + 2 * (size_t)rec_cap) +
      sizeof(int32_t) * ((size_t)sweep_cap + 2) +
      (job.want_P && !job.P_store ? sizeof(double) * (size_t)pat_stride * job.nu : 0) +
      (job.consumer == 4 || job.keep_adj ? sizeof(double) * ((size_t)4 * cap * cap + 4 * cap +
                                             (size_t)(cap + 1) * NC_MAX)
                         : 0);
  const char* env = std::getenv("MAG_SCRATCH_GB");
  const double budget_gb = env ? std::atof(env) : 8.0;
  int64_t bmax = (int64_t)(budget_gb * 1e9 / (double)per_slot);
  if (job.consumer == 4) bmax -= bmax % NORB;  // whole atoms per chunk
  if (bmax < NORB) bmax = NORB;
  return std::min(n, bmax);
}

// workgroup shapes for a nu capacity, by rows held
std::vector<KrylovShapeInfo> krylov_shape_list(int cap) {
  std::vector<KrylovShapeInfo> shapes(8);
  shapes.resize(std::min<int>(8, krylov_shapes(cap, shapes.data(), 8)));
  std::sort(shapes.begin(), shapes.end(),
            [](const KrylovShapeInfo& x, const KrylovShapeInfo& y) { return x.rows() < y.rows(); });
  return shapes;
}

// workgroup shapes for the job's nu (by rows held) and the bucket of every column
int column_buckets(mag_ctx* ctx, const ColumnJob& job, std::vector<KrylovShapeInfo>& shapes,
                   std::vector<int8_t>& bucket) {
  const int cap = krylov_capacity(job.nu);
  shapes = krylov_shape_list(cap);
  const int64_t n = (int64_t)job.cols_host.size();
  bucket.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    const int rows = NORB * ctx->h_clus_size[job.cols_host[i] >> 2];
    int b = 0;
    while (b < (int)shapes.size() && shapes[b].rows() < rows) ++b;
    if (b == (int)shapes.size())
      return fail(ctx, MAG_EUNSUPPORTED, "cluster larger than the Krylov kernel holds for this nu");
    bucket[i] = (int8_t)b;
  }
  return MAG_OK;
}

// Slot lists of one chunk: the positions [0, cnt) grouped by bucket (in
// chunk order, so each bucket stays spatially ordered), the bucket offsets,
// and each bucket's queue ranges (KRYLOV_QUEUES + 1 entries per bucket).
void chunk_lists(const mag_ctx* ctx, const int32_t* cols, const int8_t* bucket, int64_t cnt,
                 int nbk, std::vector<int32_t>& hslots, std::vector<int64_t>& hqbeg,
                 std::vector<int64_t>& boff) {
  hslots.clear();
  hqbeg.assign((size_t)(KRYLOV_QUEUES + 1) * nbk, 0);
  boff.assign(nbk + 1, 0);
  for (int b = 0; b < nbk; ++b) {
    boff[b] = (int64_t)hslots.size();
    std::vector<int32_t> bcols;
    for (int64_t q = 0; q < cnt; ++q)
      if (bucket[q] == b) {
        hslots.push_back((int32_t)q);
        bcols.push_back(cols[q]);
      }
    if (!bcols.empty()) {
      const std::vector<int64_t> qb = queue_ranges(ctx, bcols.data(), (int64_t)bcols.size());
      std::copy(qb.begin(), qb.end(), hqbeg.begin() + (size_t)(KRYLOV_QUEUES + 1) * b);
    }
  }
  boff[nbk] = (int64_t)hslots.size();
}

// device column lists of every chunk of a captured solve
struct GraphLists {
  const int32_t* slots = nullptr;  // concatenated chunk lists
  const int64_t* qbeg = nullptr;   // per (chunk, bucket): KRYLOV_QUEUES + 1
  int32_t* queue = nullptr;        // per (chunk, bucket): KRYLOV_QUEUES counters
  std::vector<std::vector<int64_t>> boff;  // host: per chunk, bucket offsets
  std::vector<int64_t> slot_base;          // host: per chunk, offset into slots
};

// ---- Krylov launch plans and their tuning

static size_t lds_per_cu(int device) {
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) !=
          hipSuccess ||
      v <= 0) {
    (void)hipGetLastError();
    v = 65536;
  }
  return (size_t)v;
}

// largest block cache for `per_cu` workgroups of a shape on one CU (0 if the
// cache is switched off or does not fit)
static size_t cache_bytes(int shape, int per_cu, int device) {
  const char* env = std::getenv("MAG_LDS_CACHE");
  if (env && std::atoi(env) == 0) return 0;
  const size_t slot = (size_t)CSLOT_BYTES;
  const long share = (long)(lds_per_cu(device) / per_cu) - (long)krylov_static_lds(shape) - 512;
  if (share < (long)slot) return 0;
  size_t dyn = ((size_t)share / slot) * slot;
  dyn = std::min(dyn, (size_t)krylov_cache_blocks((size_t)1 << 30) * slot);
  while (dyn > 0 && krylov_occupancy(shape, dyn) < per_cu) dyn -= slot;
  return dyn;
}

static KrylovPlan make_plan(int shape, int per_cu, int device) {
  KrylovPlan p;
  p.shape = shape;
  p.per_cu = per_cu;
  p.dyn = cache_bytes(shape, per_cu, device);
  p.cache = krylov_cache_blocks(p.dyn);
  return p;
}

// the plan of bucket b (default: its own shape, as many workgroups per CU as
// fit, the LDS left over as block cache)
KrylovPlan& krylov_plan(mag_ctx* ctx, const std::vector<KrylovShapeInfo>& shapes, int b, int ncu) {
  (void)ncu;
  const auto key = std::make_pair(shapes[b].cap, shapes[b].id);
  auto it = ctx->kplans.find(key);
  if (it != ctx->kplans.end()) return it->second;
  const int occ = std::max(1, krylov_occupancy(shapes[b].id, 0));
  KrylovPlan p = make_plan(shapes[b].id, occ, ctx->device);
  const char* env = std::getenv("MAG_AUTOTUNE");
  p.tuned = env && std::atoi(env) == 0;  // tuning off: keep the default
  return ctx->kplans.emplace(key, p).first->second;
}

// Time the candidate plans of bucket b -- its own shape and every larger one,
// each with 1 .. (occupancy) workgroups per CU and the largest block cache
// that leaves them -- on a sample of the bucket's columns, and keep the
// fastest.  Every candidate computes the same columns (the results do not
// depend on the plan), so the sample's outputs are simply overwritten by the
// real launch.
int krylov_tune(mag_ctx* ctx, const std::vector<KrylovShapeInfo>& shapes, int b,
                const KrylovArgs& ka, int64_t off, int64_t nb, int ncu,
                const int32_t* hslots, const int32_t* hcols) {
  KrylovPlan& plan = krylov_plan(ctx, shapes, b, ncu);
  if (plan.tuned) return MAG_OK;
  plan.tuned = true;
  if (nb < ncu) return MAG_OK;  // too few columns to fill the device: keep the default
  const int64_t S = std::min<int64_t>(nb, 4 * (int64_t)ncu);
  // queue ranges over the sample, in the spare queue slot after the buckets
  std::vector<int32_t> scols(S);
  for (int64_t i = 0; i < S; ++i) scols[i] = hcols[hslots[i]];
  const std::vector<int64_t> qb = queue_ranges(ctx, scols.data(), S);
  int64_t* dq = ctx->k_qbeg.as<int64_t>() + (KRYLOV_QUEUES + 1) * (int64_t)shapes.size();
  HIPCHK(hipMemcpyAsync(dq, qb.data(), sizeof(int64_t) * qb.size(), hipMemcpyHostToDevice,
                        ctx->stream));
  TRY(sync(ctx));
  int32_t* dc = ctx->k_queue.as<int32_t>() + KRYLOV_QUEUES * (int64_t)shapes.size();

  std::vector<KrylovPlan> cand;
  for (int s2 = 0; s2 < (int)shapes.size(); ++s2) {
    if (shapes[s2].rows() < shapes[b].rows()) continue;  // too small for the bucket
    const int occ = std::max(1, krylov_occupancy(shapes[s2].id, 0));
    for (int pc = 1; pc <= occ; ++pc) cand.push_back(make_plan(shapes[s2].id, pc, ctx->device));
  }
  plan.candidates = (int)cand.size();
  if (cand.size() < 2) return MAG_OK;  // nothing to choose
  hipEvent_t t0 = nullptr, t1 = nullptr;
  HIPCHK(hipEventCreate(&t0));
  if (hipEventCreate(&t1) != hipSuccess) {
    (void)hipEventDestroy(t0);
    return fail(ctx, MAG_EHIP, "hipEventCreate failed");
  }
  Timer tt(ctx->stream);
  double best = 1e300;
  for (const KrylovPlan& c : cand) {
    KrylovArgs kt = ka;
    kt.slots = ctx->k_slots.as<int32_t>() + off;
    kt.ncols = S;
    kt.cache_cap = c.cache;
    kt.queue = dc;
    kt.qbeg = dq;
    kt.nqueue = KRYLOV_QUEUES;
    const int grid = (int)std::min<int64_t>(S, (int64_t)ncu * c.per_cu);
    float ms = 0.f;
    for (int rep = 0; rep < 2; ++rep) {  // the first launch also loads the code object
      HIPCHK(launch_fill_i32(dc, KRYLOV_QUEUES, 0, ctx->stream));
      HIPCHK(hipEventRecord(t0, ctx->stream));
      HIPCHK(launch_krylov(kt, c.shape, c.dyn, grid, ctx->stream));
      HIPCHK(hipEventRecord(t1, ctx->stream));
      HIPCHK(hipEventSynchronize(t1));
      HIPCHK(hipEventElapsedTime(&ms, t0, t1));
    }
    const double us = 1e3 * ms / (double)S;
    if (us < best) {
      best = us;
      plan = c;
      plan.tuned = true;
      plan.us_per_col = us;
      plan.candidates = (int)cand.size();
    }
  }
  ctx->stats.autotune_ms += tt.stop_ms();
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  return MAG_OK;
}

// the plans of the pass's buckets, for mag_get_stats
static void record_plans(mag_ctx* ctx, const std::vector<KrylovShapeInfo>& shapes,
                         const std::vector<const KrylovPlan*>& plans,
                         const std::vector<int64_t>& boff) {
  mag_stats& st = ctx->stats;
  for (int b = 0; b < MAG_STATS_BUCKETS; ++b) {
    st.plan_threads[b] = st.plan_rows[b] = st.plan_per_cu[b] = 0;
    st.plan_cache[b] = st.plan_candidates[b] = 0;
    st.plan_columns[b] = 0;
    st.plan_us_per_col[b] = 0.0;
  }
  for (int b = 0; b < (int)plans.size() && b < MAG_STATS_BUCKETS; ++b) {
    if (!plans[b]) continue;
    for (const KrylovShapeInfo& sh : shapes)
      if (sh.id == plans[b]->shape) {
        st.plan_threads[b] = sh.tpb;
        st.plan_rows[b] = sh.r;
      }
    st.plan_per_cu[b] = plans[b]->per_cu;
    st.plan_cache[b] = plans[b]->cache;
    st.plan_candidates[b] = plans[b]->candidates;
    st.plan_columns[b] = boff[b + 1] - boff[b];
    st.plan_us_per_col[b] = plans[b]->us_per_col;
  }
}

// the exact gradient of one chunk of whole atoms whose pass-1 data (Ritz
// vectors, basis, h, beta, last residual) are in the adj_* buffers: the
// pencil's adjoint, the reverse sweep with the contraction, per-atom parts
static int adjoint_tail(mag_ctx* ctx, const ColumnJob& job, const int32_t* cols,
                        const int32_t* nu_eff, int64_t cnt, int cap, int ncu) {
  HIPCHK(launch_adj_prep(ctx->adj_cvec.as<double>(), ctx->adj_cdg.as<double>(), nu_eff, cnt, cap,
                         ctx->state.as<MuState>(), ctx->adj_hbar.as<double>(), ctx->stream));
  const int occ = std::max(1, adjoint_occupancy(cap));
  const int64_t natoms = cnt / NORB;
  const int grid = (int)std::min<int64_t>(natoms, (int64_t)ncu * occ);
  ALLOC(ctx->adj_wbar, adjoint_scratch_per_wg(cap) * (size_t)grid);
  ALLOC(ctx->adj_counter, sizeof(int32_t));
  HIPCHK(launch_fill_i32(ctx->adj_counter.as<int32_t>(), 1, 0, ctx->stream));
  AdjointArgs aa{};
  aa.bptr = ctx->bptr.as<int32_t>();
  aa.bcol = ctx->bcol.as<int32_t>();
  aa.bval = ctx->bval.as<double>();
  aa.clus_ptr = ctx->clus_ptr.as<int64_t>();
  aa.clus_atoms = ctx->clus_atoms.as<int32_t>();
  aa.pos = ctx->pos.as<double>();
  for (int d = 0; d < 3; ++d) aa.box[d] = ctx->cell[d];
  aa.m = job.skm;
  aa.cols = cols;
  aa.natoms = natoms;
  aa.nu = job.nu;
  aa.breakdown = job.breakdown;
  aa.hbar = ctx->adj_hbar.as<double>();
  aa.nu_eff = nu_eff;
  aa.wbar = ctx->adj_wbar.as<double>();
  aa.fJ = ctx->adj_fJ.as<double>();
  aa.counter = ctx->adj_counter.as<int32_t>();
  aa.err = ctx->errflag.as<int32_t>();
  aa.cap = cap;
  aa.q = ctx->adj_q.as<double>();
  aa.r = ctx->adj_r.as<double>();
  aa.h = ctx->adj_h.as<double>();
  aa.beta = ctx->adj_beta.as<double>();
  aa.qrows = NC_MAX;
  HIPCHK(launch_adjoint(aa, grid, ctx->stream));
  return MAG_OK;
}

int run_columns(mag_ctx* ctx, ColumnJob& job, const GraphLists* gl = nullptr) {
  const int64_t n = (int64_t)job.cols_host.size();
  if (n == 0) return MAG_OK;
  const int cap = krylov_capacity(job.nu);
  const int pat_stride = job.full ? NC_MAX : PAT_MAX;
  const int rec_cap = eig_rec_cap(cap), sweep_cap = eig_sweep_cap(cap);
  const int64_t bsz = chunk_columns(job, n);
  ALLOC(ctx->k_hs, sizeof(double) * bsz * 2 * cap * cap);
  ALLOC(ctx->k_urow, sizeof(double) * bsz * cap);
  ALLOC(ctx->k_qpat, sizeof(double) * bsz * (size_t)pat_stride * cap);
  ALLOC(ctx->k_nu, sizeof(int32_t) * bsz);
  ALLOC(ctx->k_npat, sizeof(int32_t) * bsz);
  ALLOC(ctx->k_trid, sizeof(double) * bsz * 4 * cap);
  ALLOC(ctx->k_evu, sizeof(double) * bsz * cap);
  ALLOC(ctx->k_rot, sizeof(double) * bsz * 2 * (size_t)rec_cap);
  ALLOC(ctx->k_sweep, sizeof(int32_t) * bsz * (size_t)sweep_cap);
  ALLOC(ctx->k_qlst, sizeof(int32_t) * bsz);
  ALLOC(ctx->k_fbl, sizeof(int32_t) * bsz);
  ALLOC(ctx->k_fbc, sizeof(int32_t));
  const bool adj_out = job.consumer == 4 || job.keep_adj;
  if (adj_out) {
    ALLOC(ctx->adj_cvec, sizeof(double) * bsz * cap * cap);
    ALLOC(ctx->adj_cdg, sizeof(double) * bsz * 3 * cap);
    ALLOC(ctx->adj_hbar, sizeof(double) * bsz * 2 * cap * cap);
    ALLOC(ctx->adj_q, sizeof(double) * bsz * cap * (size_t)NC_MAX);
    ALLOC(ctx->adj_r, sizeof(double) * bsz * (size_t)NC_MAX);
    ALLOC(ctx->adj_h, sizeof(double) * bsz * cap * cap);
    ALLOC(ctx->adj_beta, sizeof(double) * bsz * cap);
  }
  double* Pbuf = job.P_store;
  if (job.want_P && !job.P_store) {
    ALLOC(ctx->tmp_out, sizeof(double) * bsz * (size_t)pat_stride * job.nu);
    Pbuf = ctx->tmp_out.as<double>();
  }
  // workgroup shapes for this nu and the bucket (shape index) of every column
  std::vector<KrylovShapeInfo> shapes;
  std::vector<int8_t> bucket;
  // (a pass over every column in one chunk keeps its buckets and launch
  // lists, which the next such pass of the same system and nu reuses)
  mag_ctx::OrderLists& ol = ctx->lists;
  const bool one_chunk_order = job.order && bsz >= n;
  const bool same_order =
      one_chunk_order && ol.valid && ol.sys_gen == ctx->sys_gen && ol.cap == cap;
  if (same_order) {
    shapes = krylov_shape_list(cap);
  } else {
    TRY(column_buckets(ctx, job, shapes, bucket));
  }
  const int8_t* bkt = same_order ? ol.bucket.data() : bucket.data();
  const int nbk = (int)shapes.size();
  ALLOC(ctx->k_slots, sizeof(int32_t) * bsz);
  ALLOC(ctx->k_queue, sizeof(int32_t) * KRYLOV_QUEUES * (nbk + 1));
  ALLOC(ctx->k_qbeg, sizeof(int64_t) * (KRYLOV_QUEUES + 1) * (nbk + 1));
  // the device lists are still resident unless either buffer was allocated anew
  const bool cached = same_order && ol.slots_epoch == ctx->k_slots.epoch &&
                      ol.qbeg_epoch == ctx->k_qbeg.epoch;
  const int ncu = device_count_cus(ctx->device);
  int schedule = (job.schedule == MAG_SCHED_AUTO || job.schedule == MAG_SCHED_GRAPH)
                     ? MAG_SCHED_PERSISTENT
                     : job.schedule;
  ctx->stats.schedule_used = schedule;

  size_t timed = 0;
  for (int64_t i0 = 0; i0 < n; i0 += bsz) {
    const int64_t cnt = std::min(bsz, n - i0);

    KrylovArgs ka{};
    ka.bptr = ctx->bptr.as<int32_t>();
    ka.bcol = ctx->bcol.as<int32_t>();
    ka.bval = ctx->bval.as<double>();
    ka.clus_ptr = ctx->clus_ptr.as<int64_t>();
    ka.clus_atoms = ctx->clus_atoms.as<int32_t>();
    ka.cols = job.cols_dev + i0;
    ka.ncols = cnt;
    ka.queue = nullptr;
    ka.qbeg = nullptr;
    ka.nqueue = 0;
    ka.nu = job.nu;
    ka.breakdown = job.breakdown;
    ka.hs = ctx->k_hs.as<double>();
    ka.urow = ctx->k_urow.as<double>();
    ka.qpat = ctx->k_qpat.as<double>();
    ka.nu_eff = ctx->k_nu.as<int32_t>();
    ka.npat = ctx->k_npat.as<int32_t>();
    ka.err = ctx->errflag.as<int32_t>();
    ka.cap = cap;
    ka.pat_stride = pat_stride;
    ka.full = job.full;
    ka.cache_cap = 0;
    ka.slots = nullptr;
    if (adj_out) {  // the exact gradient reads the forward's basis back
      ka.adj_q = ctx->adj_q.as<double>();
      ka.adj_r = ctx->adj_r.as<double>();
      ka.adj_h = ctx->adj_h.as<double>();
      ka.adj_beta = ctx->adj_beta.as<double>();
      ka.adj_rows = NC_MAX;
    }

    EigArgs ea{};
    ea.hs = ka.hs;
    ea.urow = ka.urow;
    ea.qpat = ka.qpat;
    ea.nu_eff_in = ka.nu_eff;
    ea.cols = ka.cols;
    ea.rowptr = ctx->rowptr.as<int64_t>();
    ea.ncols = cnt;
    ea.cap = cap;
    ea.nu = job.nu;
    ea.eps = job.out_by_slot ? job.eps + i0 * job.nu : job.eps;
    ea.w = job.out_by_slot ? job.w + i0 * job.nu : job.w;
    ea.nu_eff_out = job.out_by_slot ? job.nu_eff + i0 : job.nu_eff;
    ea.npat = ka.npat;
    ea.P = job.want_P ? Pbuf : nullptr;
    ea.pmode = job.P_store ? 1 : 0;
    ea.pat_stride = pat_stride;
    ea.out_by_slot = job.out_by_slot;
    ea.err = ka.err;
    ea.trid = ctx->k_trid.as<double>();
    ea.evu = ctx->k_evu.as<double>();
    ea.rot = ctx->k_rot.as<double>();
    ea.sweep = ctx->k_sweep.as<int32_t>();
    ea.qlst = ctx->k_qlst.as<int32_t>();
    ea.fb_list = ctx->k_fbl.as<int32_t>();
    ea.fb_count = ctx->k_fbc.as<int32_t>();
    ea.rec_cap = rec_cap;
    ea.sweep_cap = job.eig_sweeps > 0 ? std::min(job.eig_sweeps, sweep_cap) : sweep_cap;
    ea.cvec = adj_out ? ctx->adj_cvec.as<double>() : nullptr;
    ea.cdg = adj_out ? ctx->adj_cdg.as<double>() : nullptr;

    if (schedule == MAG_SCHED_PLAIN) {
      for (int64_t q = 0; q < cnt; ++q) {
        KrylovArgs k1 = ka;
        k1.cols = ka.cols + q;
        k1.ncols = 1;
        k1.hs = ka.hs + q * 2 * cap * cap;
        k1.urow = ka.urow + q * cap;
        k1.qpat = ka.qpat + q * (int64_t)pat_stride * cap;
        k1.nu_eff = ka.nu_eff + q;
        k1.npat = ka.npat + q;
        if (ka.adj_q) {
          k1.adj_q = ka.adj_q + q * (int64_t)cap * NC_MAX;
          k1.adj_r = ka.adj_r + q * (int64_t)NC_MAX;
          k1.adj_h = ka.adj_h + q * (int64_t)cap * cap;
          k1.adj_beta = ka.adj_beta + q * (int64_t)cap;
        }
        const KrylovPlan& pl = krylov_plan(ctx, shapes, bkt[i0 + q], ncu);
        k1.cache_cap = pl.cache;
        HIPCHK(launch_krylov(k1, pl.shape, pl.dyn, 1, ctx->stream));
        EigArgs e1 = ea;
        e1.hs = k1.hs;
        e1.urow = k1.urow;
        e1.qpat = k1.qpat;
        e1.nu_eff_in = k1.nu_eff;
        e1.cols = k1.cols;
        e1.ncols = 1;
        e1.npat = k1.npat;
        if (job.out_by_slot) {
          e1.eps = ea.eps + q * job.nu;
          e1.w = ea.w + q * job.nu;
          e1.nu_eff_out = ea.nu_eff_out + q;
        }
        if (e1.P && !job.P_store) e1.P = Pbuf + q * (int64_t)pat_stride * job.nu;
        if (e1.cvec) {
          e1.cvec = ea.cvec + q * (int64_t)cap * cap;
          e1.cdg = ea.cdg + q * (int64_t)3 * cap;
        }
        HIPCHK(launch_eig(e1, ctx->stream));
      }
    } else {
      // one launch per bucket of cluster sizes, each over its own slot list
      // (spatial order kept) and, when persistent, its own queues
      std::vector<int32_t> hslots;
      std::vector<int64_t> hqbeg, boff;
      const int32_t* dslots = ctx->k_slots.as<int32_t>();
      const int64_t* dqbeg = ctx->k_qbeg.as<int64_t>();
      int32_t* dqueue = ctx->k_queue.as<int32_t>();
      std::vector<const KrylovPlan*> plans(nbk, nullptr);
      if (gl) {  // captured solve: lists are resident, plans already tuned
        const size_t c = (size_t)(i0 / bsz);
        boff = gl->boff[c];
        dslots = gl->slots + gl->slot_base[c];
        dqbeg = gl->qbeg + (int64_t)c * nbk * (KRYLOV_QUEUES + 1);
        dqueue = gl->queue + (int64_t)c * nbk * KRYLOV_QUEUES;
        for (int b = 0; b < nbk; ++b)
          if (boff[b + 1] > boff[b]) plans[b] = &krylov_plan(ctx, shapes, b, ncu);
      } else {
        // a pass over every column in one chunk with the lists of the last
        // such pass still resident: no host work, copy or synchronisation
        const int32_t* hs = nullptr;
        if (cached) {
          boff = ol.boff;
          hs = ol.hslots.data();
        } else {
          ol.valid = false;
          chunk_lists(ctx, job.cols_host.data() + i0, bkt + i0, cnt, nbk, hslots, hqbeg, boff);
          HIPCHK(hipMemcpyAsync(ctx->k_slots.p, hslots.data(), sizeof(int32_t) * hslots.size(),
                                hipMemcpyHostToDevice, ctx->stream));
          HIPCHK(hipMemcpyAsync(ctx->k_qbeg.p, hqbeg.data(), sizeof(int64_t) * hqbeg.size(),
                                hipMemcpyHostToDevice, ctx->stream));
          TRY(sync(ctx));  // the host lists may change or go out of scope
          hs = hslots.data();
          if (one_chunk_order) {
            if (!same_order) ol.bucket = bucket;  // else ol.bucket is what bkt points to
            ol.hslots = hslots;
            ol.hqbeg = hqbeg;
            ol.boff = boff;
            ol.sys_gen = ctx->sys_gen;
            ol.cap = cap;
            ol.slots_epoch = ctx->k_slots.epoch;
            ol.qbeg_epoch = ctx->k_qbeg.epoch;
            ol.valid = true;
            hs = ol.hslots.data();
          }
        }
        // plans (tuned on first use) before the timed launches
        for (int b = 0; b < nbk; ++b) {
          if (boff[b + 1] == boff[b]) continue;
          plans[b] = &krylov_plan(ctx, shapes, b, ncu);
          if (schedule == MAG_SCHED_PERSISTENT && !plans[b]->tuned)
            TRY(krylov_tune(ctx, shapes, b, ka, boff[b], boff[b + 1] - boff[b], ncu,
                            hs + boff[b], job.cols_host.data() + i0));
        }
      }
      hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
      if (ctx->time_kernels && !gl) {
        e0 = pool_event(ctx, 3 * timed + 0);
        e1 = pool_event(ctx, 3 * timed + 1);
        e2 = pool_event(ctx, 3 * timed + 2);
      }
      {
        int used = 0, tpb = 0, cache = 0;
        for (int b = 0; b < nbk; ++b)
          if (plans[b]) {
            ++used;
            cache = plans[b]->cache;
            for (const KrylovShapeInfo& sh : shapes)
              if (sh.id == plans[b]->shape) tpb = sh.tpb;
          }
        ctx->stats.krylov_buckets = used;
        ctx->stats.krylov_tpb = tpb;
        ctx->stats.krylov_cache_blocks = cache;
        record_plans(ctx, shapes, plans, boff);
      }
      if (e0) HIPCHK(hipEventRecord(e0, ctx->stream));
      for (int b = 0; b < nbk; ++b) {
        const int64_t nb = boff[b + 1] - boff[b];
        if (nb == 0) continue;
        const KrylovPlan& pl = *plans[b];
        KrylovArgs kb = ka;
        kb.slots = dslots + boff[b];
        kb.ncols = nb;
        kb.cache_cap = pl.cache;
        int grid = (int)nb;
        if (schedule == MAG_SCHED_PERSISTENT) {
          HIPCHK(launch_fill_i32(dqueue + KRYLOV_QUEUES * b, KRYLOV_QUEUES, 0, ctx->stream));
          kb.queue = dqueue + KRYLOV_QUEUES * b;
          kb.qbeg = dqbeg + (KRYLOV_QUEUES + 1) * b;
          kb.nqueue = KRYLOV_QUEUES;
          grid = (int)std::min<int64_t>(nb, (int64_t)ncu * pl.per_cu);
        }
        HIPCHK(launch_krylov(kb, pl.shape, pl.dyn, grid, ctx->stream));
      }
      if (e1) HIPCHK(hipEventRecord(e1, ctx->stream));
      HIPCHK(launch_eig(ea, ctx->stream));
      if (e2) {
        HIPCHK(hipEventRecord(e2, ctx->stream));
        ++timed;
      }
    }

    if (job.consumer == 4) TRY(adjoint_tail(ctx, job, ka.cols, ka.nu_eff, cnt, cap, ncu));
    if (job.consumer == 2) {
      HIPCHK(launch_cluster_rho(Pbuf, pat_stride, ka.cols, cnt, ka.npat, job.out_off + i0,
                                job.eps + i0 * job.nu, job.nu_eff + i0, job.nu,
                                ctx->state.as<MuState>(), job.out, ctx->stream));
    } else if (job.consumer == 3) {
      HIPCHK(launch_green(Pbuf, pat_stride, ka.cols, cnt, ka.npat, job.out_off + i0,
                          job.eps + i0 * job.nu, job.nu_eff + i0, job.nu, job.z, job.nz, job.out,
                          ctx->stream));
    }
    if (job.consumer == 1) {
      DensityArgs da{};
      da.P = Pbuf;
      da.pmode = job.P_store ? 1 : 0;
      da.pat_stride = pat_stride;
      da.cols = ka.cols;
      da.rowptr = ctx->rowptr.as<int64_t>();
      da.eps = ctx->eps.as<double>();
      da.nu_eff = ctx->nu_eff.as<int32_t>();
      da.ncols = cnt;
      da.nu = job.nu;
      da.st = ctx->state.as<MuState>();
      da.rho = job.rho;
      da.pi = job.pi;
      HIPCHK(launch_density(da, ctx->stream));
    }
    // the next chunk reuses the scratch: stream order keeps it safe
  }
  if (job.keep_adj && bsz >= n) {
    // one chunk held every column: its exact-gradient inputs stay for
    // mag_forces_exact (the column dimensions with them)
    ALLOC(ctx->adj_nu, sizeof(int32_t) * n);
    HIPCHK(hipMemcpyAsync(ctx->adj_nu.p, ctx->k_nu.p, sizeof(int32_t) * n,
                          hipMemcpyDeviceToDevice, ctx->stream));
    ctx->adj_kept = true;
  }
  if (ctx->time_kernels) ctx->timed_launches = timed;
  return MAG_OK;
}

// the per-launch Krylov and eigensolver times of the last timed pass, after
// a synchronisation
int read_kernel_times(mag_ctx* ctx) {
  const size_t timed = ctx->timed_launches;
  ctx->timed_launches = 0;
  {
    double tk = 0.0, te = 0.0;
    for (size_t q = 0; q < timed; ++q) {
      float a = 0.f, b = 0.f;
      HIPCHK(hipEventElapsedTime(&a, ctx->ev_pool[3 * q], ctx->ev_pool[3 * q + 1]));
      HIPCHK(hipEventElapsedTime(&b, ctx->ev_pool[3 * q + 1], ctx->ev_pool[3 * q + 2]));
      tk += a;
      te += b;
    }
    ctx->stats.t_krylov_ms = tk;
    ctx->stats.t_eig_ms = te;
    ctx->stats.krylov_launches = (int32_t)timed;
  }
  return MAG_OK;
}

int check_opts(mag_ctx* ctx, const mag_opts* o) {
  if (!o) return fail(ctx, MAG_EINVAL, "opts is NULL");
  if (o->nu < 1 || o->nu > NU_MAX)
    return fail(ctx, MAG_EINVAL, "nu must be in 1.." + std::to_string(NU_MAX));
  if (!(o->kT > 0.0) || !std::isfinite(o->kT)) return fail(ctx, MAG_EINVAL, "kT must be > 0");
  if (o->workflow != MAG_WORKFLOW_RECOMPUTE && o->workflow != MAG_WORKFLOW_STORE &&
      o->workflow != MAG_WORKFLOW_AUTO)
    return fail(ctx, MAG_EINVAL, "unknown workflow");
  if (o->schedule < MAG_SCHED_AUTO || o->schedule > MAG_SCHED_GRAPH)
    return fail(ctx, MAG_EINVAL, "unknown schedule");
  if (!std::isnan(o->mu_fixed) && !std::isfinite(o->mu_fixed))
    return fail(ctx, MAG_EINVAL, "mu_fixed must be finite or NaN");
  if (o->keep_exact != 0 && o->keep_exact != 1)
    return fail(ctx, MAG_EINVAL, "keep_exact must be 0 or 1");
  return MAG_OK;
}

int ensure_system(mag_ctx* ctx) {
  if (!ctx) return MAG_EINVAL;
  if (!ctx->has_system) return fail(ctx, MAG_ESTATE, "no system: call mag_set_system first");
  HIPCHK(hipSetDevice(ctx->device));
  return MAG_OK;
}

// pass 2: rho and pi on the pattern
// the synchronisation that ends a call: reads pass 2's timing and flags if
// pass 2 was enqueued in it, then the flags of the call's own kernels
// (copied by flags_enqueue(ctx, FLAGS_CALL) after them) unless where is null
int settle(mag_ctx* ctx, const char* where) {
  TRY(sync(ctx));
  if (ctx->pass2_pending) {
    ctx->pass2_pending = false;
    ctx->stats.t_pass2_ms = span_ms(ctx, SPAN_PASS2);
    TRY(flags_status(ctx, ctx->h_flags[FLAGS_PASS2], "pass 2"));
    ctx->density_ready = true;
  }
  return where ? flags_status(ctx, ctx->h_flags[FLAGS_CALL], where) : MAG_OK;
}

// rho and pi on the pattern (pass 2).  With defer, pass 2 is only enqueued:
// the caller's kernels that read rho and pi follow it in stream order, and
// the caller's settle() checks it.
int ensure_density(mag_ctx* ctx, bool defer = false) {
  if (!ctx->solved) return fail(ctx, MAG_ESTATE, "no solve: call mag_solve_columns first");
  if (ctx->density_ready) return MAG_OK;
  ALLOC(ctx->rho, sizeof(double) * ctx->nnz);
  ALLOC(ctx->pi, sizeof(double) * ctx->nnz);
  TRY(span_mark(ctx, SPAN_PASS2, 0));
  if (ctx->opts.workflow == MAG_WORKFLOW_STORE) {
    DensityArgs da{};
    da.P = ctx->P.as<double>();
    da.pmode = 1;
    da.pat_stride = PAT_MAX;
    da.cols = ctx->k_cols.as<int32_t>();
    da.rowptr = ctx->rowptr.as<int64_t>();
    da.eps = ctx->eps.as<double>();
    da.nu_eff = ctx->nu_eff.as<int32_t>();
    da.ncols = ctx->M;
    da.nu = ctx->nu;
    da.st = ctx->state.as<MuState>();
    da.rho = ctx->rho.as<double>();
    da.pi = ctx->pi.as<double>();
    HIPCHK(launch_density(da, ctx->stream));
  } else {
    ColumnJob job;
    job.cols_dev = ctx->k_cols.as<int32_t>();
    job.cols_host = ctx->h_order;
    job.order = true;
    job.nu = ctx->nu;
    job.breakdown = ctx->opts.breakdown > 0 ? ctx->opts.breakdown : 1e-12;
    job.eig_sweeps = ctx->opts.eig_sweeps;
    job.schedule = ctx->opts.schedule;
    // recomputed spectra go to scratch rows so the pass-1 data stay as they are
    ALLOC(ctx->tmp_cols, sizeof(double) * 2 * ctx->M * ctx->nu + sizeof(int32_t) * ctx->M);
    job.eps = ctx->tmp_cols.as<double>();
    job.w = job.eps + ctx->M * ctx->nu;
    job.nu_eff = reinterpret_cast<int32_t*>(job.w + ctx->M * ctx->nu);
    job.want_P = 1;
    job.consumer = 1;
    job.rho = ctx->rho.as<double>();
    job.pi = ctx->pi.as<double>();
    TRY(run_columns(ctx, job));
  }
  TRY(span_mark(ctx, SPAN_PASS2, 1));
  TRY(flags_enqueue(ctx, FLAGS_PASS2));
  ctx->pass2_pending = true;
  return defer ? MAG_OK : settle(ctx, nullptr);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int mag_version(void) { return 100; }

const char* mag_last_error(const mag_ctx* ctx) {
  if (!ctx) return "context is NULL";
  return ctx->err.c_str();
}

int mag_create(mag_ctx** out, int device, void* hip_stream) {
  if (!out) return MAG_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return MAG_EHIP;
  if (device < 0 || device >= ndev) return MAG_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return MAG_EHIP;
  mag_ctx* ctx = new mag_ctx();
  ctx->device = device;
  if (hip_stream) {
    ctx->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
      delete ctx;
      return MAG_EHIP;
    }
    ctx->own_stream = true;
  }
  noalloc_init(device);  // the allocation-free entry point's scratch address on this device
  void* hp = nullptr;
  if (hipHostMalloc(&hp, sizeof(MuState), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    mag_destroy(ctx);
    return MAG_ENOMEM;
  }
  ctx->h_state_pinned = static_cast<MuState*>(hp);
  if (hipHostMalloc(&hp, 16 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    mag_destroy(ctx);
    return MAG_ENOMEM;
  }
  ctx->h_flags = static_cast<int32_t*>(hp);
  std::fill(ctx->h_flags, ctx->h_flags + 16, 0);
  if (ctx->errflag.reserve(256) != hipSuccess || ctx->state.reserve(sizeof(MuState)) != hipSuccess ||
      hipMemset(ctx->errflag.p, 0, 256) != hipSuccess ||
      hipMemset(ctx->state.p, 0, sizeof(MuState)) != hipSuccess) {
    mag_destroy(ctx);
    return MAG_ENOMEM;
  }
  *out = ctx;
  return MAG_OK;
}

void mag_destroy(mag_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  const bool own = ctx->own_stream;
  hipStream_t s = ctx->stream;
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : ctx->ev_span) (void)hipEventDestroy(e);
  if (ctx->graph.exec) (void)hipGraphExecDestroy(ctx->graph.exec);
  if (ctx->h_state_pinned) (void)hipHostFree(ctx->h_state_pinned);
  if (ctx->h_flags) (void)hipHostFree(ctx->h_flags);
  if (ctx->aux_stream) (void)hipStreamDestroy(ctx->aux_stream);
  delete ctx;  // DevBuf destructors free device memory
  if (own && s) (void)hipStreamDestroy(s);
}

void mag_opts_default(mag_opts* o) {
  if (!o) return;
  o->nu = 30;
  o->kT = 0.1;
  o->n_electrons = 0.0;
  o->mu_tol = 1e-12;
  o->mu_fixed = std::nan("");
  o->breakdown = 1e-12;
  o->workflow = MAG_WORKFLOW_AUTO;
  o->schedule = MAG_SCHED_AUTO;
  o->eig_sweeps = 0;
  o->keep_exact = 0;
}

// ---------------------------------------------------------------------------
// Slater-Koster
// ---------------------------------------------------------------------------
int mag_sk_build(mag_ctx* ctx, const mag_sk_model* model, int64_t n_atoms, const double* pos,
                 const double cell[3], int mem_kind, int64_t* nnz_out) {
  if (!ctx) return MAG_EINVAL;
  TRY(check_mem_kind(ctx, mem_kind));
  HIPCHK(hipSetDevice(ctx->device));
  if (!model_ok(model)) return fail(ctx, MAG_EINVAL, "invalid Slater-Koster model");
  if (n_atoms < 1 || !pos || !cell) return fail(ctx, MAG_EINVAL, "need n_atoms >= 1, pos, cell");
  if ((int64_t)NORB * n_atoms > (int64_t)INT32_MAX / 2)
    return fail(ctx, MAG_EUNSUPPORTED, "too many atoms for 32-bit column indices");
  for (int d = 0; d < 3; ++d)
    if (!(cell[d] > 2.0 * model->r_cut) || !std::isfinite(cell[d]))
      return fail(ctx, MAG_EINVAL, "every box length must exceed 2 r_cut");
  ctx->sk_built = false;
  const int64_t n = n_atoms;
  TRY(copy_in(ctx, ctx->sk_pos, pos, sizeof(double) * 3 * n, mem_kind));
  HIPCHK(launch_check_finite(ctx->sk_pos.as<double>(), 3 * n, ctx->errflag.as<int32_t>(),
                             ctx->stream));
  TRY(take_errors(ctx, "mag_sk_build"));
  CellList& cl = ctx->sk_cells;
  HIPCHK(build_cell_list(cl, ctx->sk_pos.as<double>(), n, cell, model->r_cut, ctx->stream));
  DevBuf& cnt = ctx->sk_cnt;
  ALLOC(cnt, sizeof(int32_t) * n);
  HIPCHK(launch_sk_count(ctx->sk_pos.as<double>(), n, cell, model->r_cut, cl, cnt.as<int32_t>(),
                         ctx->errflag.as<int32_t>(), ctx->stream));
  std::vector<int32_t> hc(n), hb(n + 1);
  HIPCHK(hipMemcpyAsync(hc.data(), cnt.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, ctx->stream));
  TRY(take_errors(ctx, "mag_sk_build"));
  hb[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (hc[i] > BLOCKS_MAX)
      return fail(ctx, MAG_EUNSUPPORTED, "atom " + std::to_string(i) +
                                             " has more than MAG_BLOCKS_MAX pattern blocks");
    if ((int64_t)hb[i] + hc[i] > INT32_MAX / 32)
      return fail(ctx, MAG_EUNSUPPORTED, "too many blocks");
    hb[i + 1] = hb[i] + hc[i];
  }
  const int64_t nblk = hb[n];
  const int64_t nnz = 16 * nblk;
  ALLOC(ctx->sk_bptr, sizeof(int32_t) * (n + 1));
  ALLOC(ctx->sk_bcol, sizeof(int32_t) * nblk);
  ALLOC(ctx->sk_rowptr, sizeof(int64_t) * (NORB * n + 1));
  ALLOC(ctx->sk_colind, sizeof(int32_t) * nnz);
  ALLOC(ctx->sk_H, sizeof(double) * nnz);
  ALLOC(ctx->sk_S, sizeof(double) * nnz);
  HIPCHK(hipMemcpyAsync(ctx->sk_bptr.p, hb.data(), sizeof(int32_t) * (n + 1),
                        hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(launch_sk_fill(ctx->sk_pos.as<double>(), n, cell, model->r_cut, cl,
                        ctx->sk_bptr.as<int32_t>(), ctx->sk_bcol.as<int32_t>(), ctx->stream));
  HIPCHK(launch_sk_csr(ctx->sk_bptr.as<int32_t>(), ctx->sk_bcol.as<int32_t>(), n,
                       ctx->sk_rowptr.as<int64_t>(), ctx->sk_colind.as<int32_t>(), ctx->stream));
  ctx->sk_model = to_dev(*model);
  HIPCHK(launch_sk_values(ctx->sk_model, ctx->sk_pos.as<double>(), n, cell,
                          ctx->sk_bptr.as<int32_t>(), ctx->sk_bcol.as<int32_t>(),
                          ctx->sk_H.as<double>(), ctx->sk_S.as<double>(), ctx->stream));
  TRY(take_errors(ctx, "mag_sk_build"));
  ctx->sk_built = true;
  ctx->sk_n = n;
  ctx->sk_nnz = nnz;
  ctx->sk_nblk = nblk;
  for (int d = 0; d < 3; ++d) ctx->sk_cell[d] = cell[d];
  if (nnz_out) *nnz_out = nnz;
  return MAG_OK;
}

int mag_sk_get_csr(mag_ctx* ctx, int64_t* rowptr, int32_t* colind, double* H, double* S,
                   int mem_kind) {
  if (!ctx) return MAG_EINVAL;
  TRY(check_mem_kind(ctx, mem_kind));
  if (!ctx->sk_built) return fail(ctx, MAG_ESTATE, "no Slater-Koster build");
  HIPCHK(hipSetDevice(ctx->device));
  TRY(copy_out(ctx, rowptr, ctx->sk_rowptr.p, sizeof(int64_t) * (NORB * ctx->sk_n + 1), mem_kind));
  TRY(copy_out(ctx, colind, ctx->sk_colind.p, sizeof(int32_t) * ctx->sk_nnz, mem_kind));
  TRY(copy_out(ctx, H, ctx->sk_H.p, sizeof(double) * ctx->sk_nnz, mem_kind));
  TRY(copy_out(ctx, S, ctx->sk_S.p, sizeof(double) * ctx->sk_nnz, mem_kind));
  return sync(ctx);
}

int mag_sk_values(mag_ctx* ctx, const double* pos, double* H, double* S, int mem_kind) {
  if (!ctx) return MAG_EINVAL;
  TRY(check_mem_kind(ctx, mem_kind));
  if (!ctx->sk_built) return fail(ctx, MAG_ESTATE, "no Slater-Koster build");
  if (!pos) return fail(ctx, MAG_EINVAL, "pos is NULL");
  HIPCHK(hipSetDevice(ctx->device));
  TRY(copy_in(ctx, ctx->sk_pos, pos, sizeof(double) * 3 * ctx->sk_n, mem_kind));
  HIPCHK(launch_check_finite(ctx->sk_pos.as<double>(), 3 * ctx->sk_n, ctx->errflag.as<int32_t>(),
                             ctx->stream));
  HIPCHK(launch_sk_values(ctx->sk_model, ctx->sk_pos.as<double>(), ctx->sk_n, ctx->sk_cell,
                          ctx->sk_bptr.as<int32_t>(), ctx->sk_bcol.as<int32_t>(),
                          ctx->sk_H.as<double>(), ctx->sk_S.as<double>(), ctx->stream));
  TRY(take_errors(ctx, "mag_sk_values"));
  TRY(copy_out(ctx, H, ctx->sk_H.p, sizeof(double) * ctx->sk_nnz, mem_kind));
  TRY(copy_out(ctx, S, ctx->sk_S.p, sizeof(double) * ctx->sk_nnz, mem_kind));
  return sync(ctx);
}

int mag_sk_vjp(mag_ctx* ctx, const double* pos, const double* gH, const double* gS, double* grad,
               int mem_kind) {
  if (!ctx) return MAG_EINVAL;
  TRY(check_mem_kind(ctx, mem_kind));
  if (!ctx->sk_built) return fail(ctx, MAG_ESTATE, "no Slater-Koster build");
  if (!pos || !gH || !gS || !grad) return fail(ctx, MAG_EINVAL, "NULL argument");
  HIPCHK(hipSetDevice(ctx->device));
  const int64_t n = ctx->sk_n, nnz = ctx->sk_nnz;
  TRY(copy_in(ctx, ctx->sk_pos, pos, sizeof(double) * 3 * n, mem_kind));
  DevBuf bt, dgh, dgs, dgr;
  ALLOC(bt, sizeof(int32_t) * ctx->sk_nblk);
  HIPCHK(launch_block_transpose(ctx->sk_bptr.as<int32_t>(), ctx->sk_bcol.as<int32_t>(), n,
                                bt.as<int32_t>(), ctx->errflag.as<int32_t>(), ctx->stream));
  TRY(take_errors(ctx, "mag_sk_vjp"));  // every block needs its transpose before the contraction
  const double* pgh = gH;
  const double* pgs = gS;
  if (mem_kind == MAG_HOST) {
    TRY(copy_in(ctx, dgh, gH, sizeof(double) * nnz, MAG_HOST));
    TRY(copy_in(ctx, dgs, gS, sizeof(double) * nnz, MAG_HOST));
    pgh = dgh.as<double>();
    pgs = dgs.as<double>();
  }
  ALLOC(dgr, sizeof(double) * 3 * n);
  ALLOC(ctx->f_part, sizeof(double) * 3 * std::max<int64_t>(ctx->sk_nblk, 1));
  HIPCHK(launch_sk_vjp(ctx->sk_model, ctx->sk_pos.as<double>(), n, ctx->sk_nblk, ctx->sk_cell,
                       ctx->sk_bptr.as<int32_t>(), ctx->sk_bcol.as<int32_t>(), bt.as<int32_t>(),
                       pgh, pgs, 1.0, ctx->f_part.as<double>(), dgr.as<double>(), ctx->stream));
  TRY(take_errors(ctx, "mag_sk_vjp"));
  TRY(copy_out(ctx, grad, dgr.p, sizeof(double) * 3 * n, mem_kind));
  return sync(ctx);
}

// ---------------------------------------------------------------------------
// system
// ---------------------------------------------------------------------------
// a device allocation on `device` holds [p, p + bytes)
static bool device_span(const void* p, size_t bytes, int device) {
  hipPointerAttribute_t at{};
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (at.type != hipMemoryTypeDevice || at.device != device) return false;
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return (const char*)p + bytes <= (const char*)base + size;
}

int mag_sk_vjp_noalloc(mag_ctx* ctx, const double* pos, const double* gH, const double* gS,
                       double* grad) {
  if (!ctx) return MAG_EINVAL;
  if (!ctx->sk_built) return fail(ctx, MAG_ESTATE, "no Slater-Koster build");
  if (!pos || !gH || !gS || !grad) return fail(ctx, MAG_EINVAL, "NULL argument");
  const int64_t n = ctx->sk_n, nnz = ctx->sk_nnz, nblk = ctx->sk_nblk;
  if (nblk > NOALLOC_MAX_BLOCKS)
    return fail(ctx, MAG_EUNSUPPORTED,
                "the pattern has " + std::to_string(nblk) +
                    " blocks; the allocation-free path holds at most " +
                    std::to_string(NOALLOC_MAX_BLOCKS));
  HIPCHK(hipSetDevice(ctx->device));
  if (!device_span(pos, sizeof(double) * 3 * n, ctx->device) ||
      !device_span(gH, sizeof(double) * nnz, ctx->device) ||
      !device_span(gS, sizeof(double) * nnz, ctx->device) ||
      !device_span(grad, sizeof(double) * 3 * n, ctx->device))
    return fail(ctx, MAG_EINVAL,
                "pos, gH, gS and grad must be device memory of the documented sizes on the "
                "context's device");
  void* base = nullptr;
  HIPCHK(noalloc_scratch(ctx->device, &base));
  double* part = static_cast<double*>(base);
  int32_t* bt = reinterpret_cast<int32_t*>(part + 3 * NOALLOC_MAX_BLOCKS);
  HIPCHK(launch_block_transpose(ctx->sk_bptr.as<int32_t>(), ctx->sk_bcol.as<int32_t>(), n, bt,
                                ctx->errflag.as<int32_t>(), ctx->stream));
  TRY(take_errors(ctx, "mag_sk_vjp_noalloc"));  // every block needs its transpose first
  HIPCHK(launch_sk_vjp(ctx->sk_model, pos, n, nblk, ctx->sk_cell, ctx->sk_bptr.as<int32_t>(),
                       ctx->sk_bcol.as<int32_t>(), bt, gH, gS, 1.0, part, grad, ctx->stream));
  TRY(take_errors(ctx, "mag_sk_vjp_noalloc"));
  return sync(ctx);
}

int mag_set_system(mag_ctx* ctx, const mag_system* sys, int mem_kind) {
  if (!ctx) return MAG_EINVAL;
  TRY(check_mem_kind(ctx, mem_kind));
  HIPCHK(hipSetDevice(ctx->device));
  ctx->lists.valid = false;  // the column order and clusters change
  if (!sys || sys->n_atoms < 1 || sys->nnz < 1 || !sys->rowptr || !sys->colind || !sys->H ||
      !sys->S)
    return fail(ctx, MAG_EINVAL, "system needs n_atoms, nnz, rowptr, colind, H and S");
  Timer tm(ctx->stream);
  ctx->has_system = false;
  ctx->solved = false;
  ctx->density_ready = false;
  ctx->adj_kept = false;
  const int64_t N = sys->n_atoms, M = NORB * N, nnz = sys->nnz;
  if (M > (int64_t)INT32_MAX / 2)
    return fail(ctx, MAG_EUNSUPPORTED, "too many atoms for 32-bit column indices");

  // row pointers: host copy and block-complete checks
  ctx->h_rowptr.assign(M + 1, 0);
  HIPCHK(hipMemcpyAsync(ctx->h_rowptr.data(), sys->rowptr, sizeof(int64_t) * (M + 1),
                        mem_kind == MAG_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost,
                        ctx->stream));
  TRY(sync(ctx));
  const std::vector<int64_t>& rp = ctx->h_rowptr;
  if (rp[0] != 0 || rp[M] != nnz) return fail(ctx, MAG_EINVAL, "rowptr[0] != 0 or rowptr[M] != nnz");
  std::vector<int32_t> hb(N + 1);
  ctx->h_bcount.assign(N, 0);
  hb[0] = 0;
  for (int64_t J = 0; J < N; ++J) {
    const int64_t len = rp[NORB * J + 1] - rp[NORB * J];
    if (len <= 0 || len % NORB != 0 || len / NORB > BLOCKS_MAX)
      return fail(ctx, MAG_EINVAL, "row " + std::to_string(NORB * J) +
                                       ": length not a positive multiple of 4 within the block limit");
    for (int a = 1; a < NORB; ++a)
      if (rp[NORB * J + a + 1] - rp[NORB * J + a] != len)
        return fail(ctx, MAG_EINVAL, "rows of atom " + std::to_string(J) + " differ in length");
    if (rp[NORB * J] != 16 * (int64_t)hb[J])
      return fail(ctx, MAG_EINVAL, "CSR is not block-complete at atom " + std::to_string(J));
    ctx->h_bcount[J] = (int32_t)(len / NORB);
    if ((int64_t)hb[J] + len / NORB > INT32_MAX / 32) return fail(ctx, MAG_EUNSUPPORTED, "too many blocks");
    hb[J + 1] = hb[J] + (int32_t)(len / NORB);
  }
  const int64_t nblk = hb[N];
  TRY(copy_in(ctx, ctx->rowptr, sys->rowptr, sizeof(int64_t) * (M + 1), mem_kind));
  ALLOC(ctx->bptr, sizeof(int32_t) * (N + 1));
  HIPCHK(hipMemcpyAsync(ctx->bptr.p, hb.data(), sizeof(int32_t) * (N + 1), hipMemcpyHostToDevice,
                        ctx->stream));
  ALLOC(ctx->bcol, sizeof(int32_t) * nblk);
  ALLOC(ctx->btrans, sizeof(int32_t) * nblk);
  ALLOC(ctx->bval, sizeof(double) * nblk * 32);
  {
    DevBuf ci, hv, sv;
    const int32_t* pci = sys->colind;
    const double* phv = sys->H;
    const double* psv = sys->S;
    if (mem_kind == MAG_HOST) {
      TRY(copy_in(ctx, ci, sys->colind, sizeof(int32_t) * nnz, MAG_HOST));
      TRY(copy_in(ctx, hv, sys->H, sizeof(double) * nnz, MAG_HOST));
      TRY(copy_in(ctx, sv, sys->S, sizeof(double) * nnz, MAG_HOST));
      pci = ci.as<int32_t>();
      phv = hv.as<double>();
      psv = sv.as<double>();
    }
    HIPCHK(launch_check_layout(ctx->rowptr.as<int64_t>(), pci, N, ctx->bptr.as<int32_t>(),
                               ctx->bcol.as<int32_t>(), ctx->errflag.as<int32_t>(), ctx->stream));
    HIPCHK(launch_check_finite(phv, nnz, ctx->errflag.as<int32_t>(), ctx->stream));
    HIPCHK(launch_check_finite(psv, nnz, ctx->errflag.as<int32_t>(), ctx->stream));
    HIPCHK(launch_to_blocks(ctx->rowptr.as<int64_t>(), phv, psv, N, ctx->bptr.as<int32_t>(),
                            ctx->bval.as<double>(), ctx->stream));
    TRY(take_errors(ctx, "mag_set_system"));
  }
  HIPCHK(launch_block_transpose(ctx->bptr.as<int32_t>(), ctx->bcol.as<int32_t>(), N,
                                ctx->btrans.as<int32_t>(), ctx->errflag.as<int32_t>(),
                                ctx->stream));

  for (int d = 0; d < 3; ++d) ctx->cell[d] = sys->cell[d];
  ctx->r_cluster = sys->r_cluster;
  ctx->has_pos = sys->pos != nullptr;
  if (ctx->has_pos) {
    TRY(copy_in(ctx, ctx->pos, sys->pos, sizeof(double) * 3 * N, mem_kind));
    HIPCHK(launch_check_finite(ctx->pos.as<double>(), 3 * N, ctx->errflag.as<int32_t>(),
                               ctx->stream));
  }
  TRY(take_errors(ctx, "mag_set_system"));  // the transpose's and the positions' checks

  // clusters
  std::vector<int64_t> cptr(N + 1);
  std::vector<double> hp;  // positions on the host for the column order, when copied early
  if (sys->clus_ptr && sys->clus_atoms) {
    HIPCHK(hipMemcpyAsync(cptr.data(), sys->clus_ptr, sizeof(int64_t) * (N + 1),
                          mem_kind == MAG_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost,
                          ctx->stream));
    TRY(sync(ctx));
    if (cptr[0] != 0) return fail(ctx, MAG_EINVAL, "clus_ptr[0] != 0");
    for (int64_t J = 0; J < N; ++J) {
      const int64_t c = cptr[J + 1] - cptr[J];
      if (c < 1) return fail(ctx, MAG_EINVAL, "empty cluster");
      if (c > CLUSTER_MAX) return fail(ctx, MAG_EUNSUPPORTED, "cluster above MAG_CLUSTER_MAX atoms");
    }
    std::vector<int32_t> hat(cptr[N]);
    HIPCHK(hipMemcpyAsync(hat.data(), sys->clus_atoms, sizeof(int32_t) * cptr[N],
                          mem_kind == MAG_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost,
                          ctx->stream));
    TRY(sync(ctx));
    for (int64_t J = 0; J < N; ++J) {
      bool self = false;
      for (int64_t a = cptr[J]; a < cptr[J + 1]; ++a) {
        if (hat[a] < 0 || hat[a] >= N || (a > cptr[J] && hat[a] <= hat[a - 1]))
          return fail(ctx, MAG_EINVAL, "cluster lists must be ascending atom ids < N");
        self |= hat[a] == J;
      }
      if (!self) return fail(ctx, MAG_EINVAL, "every cluster must contain its own atom");
    }
    TRY(copy_in(ctx, ctx->clus_ptr, cptr.data(), sizeof(int64_t) * (N + 1), MAG_HOST));
    TRY(copy_in(ctx, ctx->clus_atoms, hat.data(), sizeof(int32_t) * cptr[N], MAG_HOST));
    TRY(sync(ctx));
  } else if (whole_cell(sys->cell, sys->r_cluster)) {
    if (N > CLUSTER_MAX)
      return fail(ctx, MAG_EUNSUPPORTED, "whole-cell cluster above MAG_CLUSTER_MAX atoms");
    std::vector<int32_t> at(N * N);
    for (int64_t J = 0; J <= N; ++J) cptr[J] = J * N;
    for (int64_t J = 0; J < N; ++J)
      for (int64_t I = 0; I < N; ++I) at[J * N + I] = (int32_t)I;
    TRY(copy_in(ctx, ctx->clus_ptr, cptr.data(), sizeof(int64_t) * (N + 1), MAG_HOST));
    TRY(copy_in(ctx, ctx->clus_atoms, at.data(), sizeof(int32_t) * N * N, MAG_HOST));
    TRY(sync(ctx));
  } else {
    if (!ctx->has_pos) return fail(ctx, MAG_EINVAL, "clusters need pos (or clus_ptr/clus_atoms)");
    CellList& cl = ctx->sys_cells;
    HIPCHK(build_cell_list(cl, ctx->pos.as<double>(), N, sys->cell, sys->r_cluster, ctx->stream));
    DevBuf& tmp = ctx->sys_tmp;
    DevBuf& cnt = ctx->sys_cnt;
    ALLOC(tmp, sizeof(int32_t) * N * (size_t)CLUSTER_MAX);
    ALLOC(cnt, sizeof(int32_t) * N);
    HIPCHK(launch_cluster_scan_cv(ctx->pos.as<double>(), N, sys->cell, sys->r_cluster, cl,
                                  tmp.as<int32_t>(), cnt.as<int32_t>(), ctx->errflag.as<int32_t>(),
                                  ctx->stream));
    std::vector<int32_t> hc(N);
    HIPCHK(hipMemcpyAsync(hc.data(), cnt.p, sizeof(int32_t) * N, hipMemcpyDeviceToHost,
                          ctx->stream));
    if (mem_kind == MAG_DEVICE) {  // the column order needs them: one round trip for both
      hp.resize(3 * N);
      HIPCHK(hipMemcpyAsync(hp.data(), ctx->pos.p, sizeof(double) * 3 * N, hipMemcpyDeviceToHost,
                            ctx->stream));
    }
    TRY(take_errors(ctx, "cluster build"));
    cptr[0] = 0;
    for (int64_t J = 0; J < N; ++J) cptr[J + 1] = cptr[J] + hc[J];
    TRY(copy_in(ctx, ctx->clus_ptr, cptr.data(), sizeof(int64_t) * (N + 1), MAG_HOST));
    ALLOC(ctx->clus_atoms, sizeof(int32_t) * std::max<int64_t>(cptr[N], 1));
    HIPCHK(launch_cluster_compact(tmp.as<int32_t>(), cnt.as<int32_t>(), ctx->clus_ptr.as<int64_t>(),
                                  N, ctx->clus_atoms.as<int32_t>(), ctx->stream));
    // cptr stays alive until the synchronisation after the column order
  }
  ctx->clus_total = cptr[N];
  ctx->h_clus_size.assign(N, 0);
  int64_t maxc = 0;
  for (int64_t J = 0; J < N; ++J) {
    ctx->h_clus_size[J] = (int32_t)(cptr[J + 1] - cptr[J]);
    maxc = std::max<int64_t>(maxc, ctx->h_clus_size[J]);
  }
  // nonzeros of every cluster, read back with the column order's upload below
  DevBuf& nz = ctx->sys_nz;
  ALLOC(nz, sizeof(int64_t) * N);
  HIPCHK(launch_cluster_nnz(ctx->bptr.as<int32_t>(), ctx->bcol.as<int32_t>(),
                            ctx->clus_ptr.as<int64_t>(), ctx->clus_atoms.as<int32_t>(), N,
                            nz.as<int64_t>(), ctx->stream));
  std::vector<int64_t> hn(N);
  HIPCHK(hipMemcpyAsync(hn.data(), nz.p, sizeof(int64_t) * N, hipMemcpyDeviceToHost, ctx->stream));

  // column order: atoms along a Morton curve of their positions (spatially
  // compact work queues), the four columns of an atom together
  std::vector<int32_t> atoms(N);
  std::iota(atoms.begin(), atoms.end(), 0);
  if (sys->pos && mem_kind == MAG_HOST) {
    const double* p = sys->pos;
    std::vector<uint64_t> key(N);
    for (int64_t i = 0; i < N; ++i) {
      uint64_t code = 0;
      uint32_t c[3];
      for (int d = 0; d < 3; ++d) {
        double f = sys->cell[d] > 0 ? p[3 * i + d] / sys->cell[d] : 0.0;
        f -= std::floor(f);
        c[d] = (uint32_t)std::min(1023.0, std::max(0.0, f * 1024.0));
      }
      for (int b = 9; b >= 0; --b)
        for (int d = 0; d < 3; ++d) code = (code << 1) | ((c[d] >> b) & 1u);
      key[i] = code;
    }
    std::stable_sort(atoms.begin(), atoms.end(),
                     [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  } else if (ctx->has_pos) {
    if (hp.size() != (size_t)(3 * N)) {
      hp.resize(3 * N);
      HIPCHK(hipMemcpyAsync(hp.data(), ctx->pos.p, sizeof(double) * 3 * N, hipMemcpyDeviceToHost,
                            ctx->stream));
      TRY(sync(ctx));
    }
    std::vector<uint64_t> key(N);
    for (int64_t i = 0; i < N; ++i) {
      uint64_t code = 0;
      uint32_t c[3];
      for (int d = 0; d < 3; ++d) {
        double f = sys->cell[d] > 0 ? hp[3 * i + d] / sys->cell[d] : 0.0;
        f -= std::floor(f);
        c[d] = (uint32_t)std::min(1023.0, std::max(0.0, f * 1024.0));
      }
      for (int b = 9; b >= 0; --b)
        for (int d = 0; d < 3; ++d) code = (code << 1) | ((c[d] >> b) & 1u);
      key[i] = code;
    }
    std::stable_sort(atoms.begin(), atoms.end(),
                     [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  }
  ctx->h_order.resize(M);
  for (int64_t i = 0; i < N; ++i)
    for (int a = 0; a < NORB; ++a) ctx->h_order[NORB * i + a] = NORB * atoms[i] + a;
  TRY(copy_in(ctx, ctx->k_cols, ctx->h_order.data(), sizeof(int32_t) * M, MAG_HOST));
  TRY(sync(ctx));
  ctx->sum_cluster_nnz = std::accumulate(hn.begin(), hn.end(), (int64_t)0);

  ctx->N = N;
  ctx->M = M;
  ctx->nnz = nnz;
  ctx->nblk = nblk;
  ctx->has_system = true;
  ++ctx->sys_gen;  // captured solves of the previous system are stale
  ctx->stats.n_columns = M;
  ctx->stats.max_cluster = NORB * maxc;
  ctx->stats.sum_cluster_nnz = ctx->sum_cluster_nnz;
  ctx->stats.t_set_system_ms = tm.stop_ms();
  return MAG_OK;
}

int mag_update_values(mag_ctx* ctx, const double* H, const double* S, int mem_kind) {
  TRY(ensure_system(ctx));
  TRY(check_mem_kind(ctx, mem_kind));
  ctx->adj_kept = false;
  if (!H || !S) return fail(ctx, MAG_EINVAL, "H and S are required");
  DevBuf hv, sv;
  const double* phv = H;
  const double* psv = S;
  if (mem_kind == MAG_HOST) {
    TRY(copy_in(ctx, hv, H, sizeof(double) * ctx->nnz, MAG_HOST));
    TRY(copy_in(ctx, sv, S, sizeof(double) * ctx->nnz, MAG_HOST));
    phv = hv.as<double>();
    psv = sv.as<double>();
  }
  HIPCHK(launch_check_finite(phv, ctx->nnz, ctx->errflag.as<int32_t>(), ctx->stream));
  HIPCHK(launch_check_finite(psv, ctx->nnz, ctx->errflag.as<int32_t>(), ctx->stream));
  HIPCHK(launch_to_blocks(ctx->rowptr.as<int64_t>(), phv, psv, ctx->N, ctx->bptr.as<int32_t>(),
                          ctx->bval.as<double>(), ctx->stream));
  TRY(take_errors(ctx, "mag_update_values"));
  ctx->solved = false;
  ctx->density_ready = false;
  return MAG_OK;
}

int mag_get_clusters(mag_ctx* ctx, int64_t* clus_ptr, int32_t* clus_atoms, int64_t* total_out,
                     int mem_kind) {
  TRY(ensure_system(ctx));
  TRY(check_mem_kind(ctx, mem_kind));
  if (total_out) *total_out = ctx->clus_total;
  TRY(copy_out(ctx, clus_ptr, ctx->clus_ptr.p, sizeof(int64_t) * (ctx->N + 1), mem_kind));
  TRY(copy_out(ctx, clus_atoms, ctx->clus_atoms.p, sizeof(int32_t) * ctx->clus_total, mem_kind));
  return sync(ctx);
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
// bisection launches for brackets up to 1e7 eV wide at tolerance tol (five
// levels per launch); launches after convergence return at once
static int mu_rounds(double tol) {
  const int levels = (int)std::ceil(std::log2(1e7 / tol)) + 2;
  return (levels + mu_levels_per_round() - 1) / mu_levels_per_round();
}

static int mu_grid(const mag_ctx* ctx) {
  // about 16 Ritz terms per thread, at most two blocks per CU: a launch is
  // short, and its tail (the last block reading every block's partials
  // back from L2) grows with the grid, so fewer, fuller blocks finish first
  // (0.58 -> 0.37 ms for the ten launches of a 15,568-column solve)
  return (int)std::min<int64_t>(512, std::max<int64_t>(1, (ctx->M * ctx->nu + 4095) / 4096));
}

// enqueue the bisection for mu and the energy sums (no host synchronisation)
static int enqueue_mu(mag_ctx* ctx, const mag_opts* opts, bool fixed) {
  const int64_t M = ctx->M;
  const int nu = ctx->nu;
  const int grid = mu_grid(ctx);
  ALLOC(ctx->partials, sizeof(double) * 64 * (size_t)grid);
  MuState* st = ctx->state.as<MuState>();
  const double tol = opts->mu_tol > 0 ? opts->mu_tol : 1e-12;
  HIPCHK(launch_mu_setup(st, opts->n_electrons, opts->kT, tol, opts->mu_fixed, fixed ? 1 : 0,
                         ctx->stream));
  if (!fixed) {
    HIPCHK(launch_mu_init(ctx->eps.as<double>(), ctx->w.as<double>(), ctx->nu_eff.as<int32_t>(),
                          M, nu, st, ctx->partials.as<double>(), grid, ctx->stream));
    const int rounds = mu_rounds(tol);
    for (int r = 0; r < rounds; ++r)
      HIPCHK(launch_mu_round(ctx->eps.as<double>(), ctx->w.as<double>(),
                             ctx->nu_eff.as<int32_t>(), M, nu, st, ctx->partials.as<double>(),
                             grid, ctx->stream));
  }
  HIPCHK(launch_energy(ctx->eps.as<double>(), ctx->w.as<double>(), ctx->nu_eff.as<int32_t>(), M,
                       nu, st, ctx->partials.as<double>(), grid, ctx->stream));
  return MAG_OK;
}

// checks and outputs once ctx->h_state holds the final state
static int finish_solve(mag_ctx* ctx, const mag_opts* opts, bool fixed, double* mu,
                        double* E_band, double* A_free) {
  ctx->stats.bisect_levels = ctx->h_state.levels;
  if (ctx->h_state.err & KERR_NONFINITE) return fail(ctx, MAG_ENONFINITE, "non-finite Ritz data");
  if (!fixed && !ctx->h_state.done)
    return fail(ctx, MAG_EBRACKET, "bisection did not reach the tolerance");
  if (!std::isfinite(ctx->h_state.E) || !std::isfinite(ctx->h_state.mu))
    return fail(ctx, MAG_ENONFINITE, "non-finite energy");
  ctx->solved = true;
  if (mu) *mu = ctx->h_state.mu;
  if (E_band) *E_band = ctx->h_state.E;
  if (A_free) *A_free = ctx->h_state.E - opts->kT * ctx->h_state.S_ent;
  return MAG_OK;
}

static bool same_opts(const mag_opts& a, const mag_opts& b) {
  auto same = [](double x, double y) { return x == y || (std::isnan(x) && std::isnan(y)); };
  return a.nu == b.nu && same(a.kT, b.kT) && same(a.n_electrons, b.n_electrons) &&
         same(a.mu_tol, b.mu_tol) && same(a.mu_fixed, b.mu_fixed) &&
         same(a.breakdown, b.breakdown) && a.workflow == b.workflow;
}

static bool graph_usable(const mag_ctx* ctx, const mag_opts& resolved) {
  const auto& g = ctx->graph;
  return g.exec && g.alloc_gen == ctx->alloc_gen && g.sys_gen == ctx->sys_gen &&
         same_opts(g.key, resolved);
}

// Capture the forward solve just run eagerly (all buffers sized, plans tuned):
// pass 1 over every chunk, the bisection and the energies, and the copy of
// the final state to pinned host memory.  Host-side column lists of the
// persistent launches are uploaded beforehand into buffers the graph owns.
static int capture_solve(mag_ctx* ctx, ColumnJob& job, const mag_opts* opts, bool fixed) {
  auto& g = ctx->graph;
  if (g.exec) {
    (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
  }
  job.schedule = MAG_SCHED_PERSISTENT;
  const int64_t n = (int64_t)job.cols_host.size();
  const int64_t bsz = chunk_columns(job, n);
  std::vector<KrylovShapeInfo> shapes;
  std::vector<int8_t> bucket;
  TRY(column_buckets(ctx, job, shapes, bucket));
  const int nbk = (int)shapes.size();
  GraphLists gl;
  std::vector<int32_t> all_slots;
  std::vector<int64_t> all_qbeg;
  for (int64_t i0 = 0; i0 < n; i0 += bsz) {
    const int64_t cnt = std::min(bsz, n - i0);
    std::vector<int32_t> hs;
    std::vector<int64_t> hq, bo;
    chunk_lists(ctx, job.cols_host.data() + i0, bucket.data() + i0, cnt, nbk, hs, hq, bo);
    gl.slot_base.push_back((int64_t)all_slots.size());
    gl.boff.push_back(bo);
    all_slots.insert(all_slots.end(), hs.begin(), hs.end());
    all_qbeg.insert(all_qbeg.end(), hq.begin(), hq.end());
  }
  const int64_t nchunks = (int64_t)gl.boff.size();
  ALLOC(g.slots, sizeof(int32_t) * std::max<size_t>(1, all_slots.size()));
  ALLOC(g.qbeg, sizeof(int64_t) * std::max<size_t>(1, all_qbeg.size()));
  ALLOC(g.queue, sizeof(int32_t) * KRYLOV_QUEUES * nbk * nchunks);
  HIPCHK(hipMemcpyAsync(g.slots.p, all_slots.data(), sizeof(int32_t) * all_slots.size(),
                        hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(g.qbeg.p, all_qbeg.data(), sizeof(int64_t) * all_qbeg.size(),
                        hipMemcpyHostToDevice, ctx->stream));
  TRY(sync(ctx));
  gl.slots = g.slots.as<int32_t>();
  gl.qbeg = g.qbeg.as<int64_t>();
  gl.queue = g.queue.as<int32_t>();
  const uint64_t gen_before = ctx->alloc_gen;

  HIPCHK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeRelaxed));
  ctx->time_kernels = false;
  int rc = run_columns(ctx, job, &gl);
  if (rc == MAG_OK) rc = enqueue_mu(ctx, opts, fixed);
  hipError_t ce = hipSuccess;
  if (rc == MAG_OK)
    ce = hipMemcpyAsync(ctx->h_state_pinned, ctx->state.p, sizeof(MuState),
                        hipMemcpyDeviceToHost, ctx->stream);
  hipGraph_t graph = nullptr;
  const hipError_t ee = hipStreamEndCapture(ctx->stream, &graph);
  if (rc != MAG_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (ce != hipSuccess || ee != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return fail(ctx, MAG_EHIP, "capture of the forward solve failed");
  }
  const hipError_t ie = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) {
    g.exec = nullptr;
    (void)hipGetLastError();
    return fail(ctx, MAG_EHIP, "instantiation of the forward solve graph failed");
  }
  if (ctx->alloc_gen != gen_before) {  // a buffer moved while capturing: do not keep it
    (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    return MAG_OK;
  }
  g.alloc_gen = ctx->alloc_gen;
  g.sys_gen = ctx->sys_gen;
  g.key = ctx->opts;
  return MAG_OK;
}

// replay of a captured forward solve
static int replay_solve(mag_ctx* ctx, const mag_opts* opts, bool fixed, double* mu,
                        double* E_band, double* A_free) {
  TRY(span_mark(ctx, SPAN_PASS1, 0));
  HIPCHK(hipGraphLaunch(ctx->graph.exec, ctx->stream));
  TRY(span_mark(ctx, SPAN_PASS1, 1));
  TRY(flags_enqueue(ctx, FLAGS_PASS1));
  TRY(sync(ctx));
  ctx->stats.t_pass1_ms = span_ms(ctx, SPAN_PASS1);
  ctx->stats.t_krylov_ms = 0.0;
  ctx->stats.t_eig_ms = 0.0;
  ctx->stats.krylov_launches = 0;
  ctx->stats.t_mu_ms = 0.0;
  ctx->stats.schedule_used = MAG_SCHED_GRAPH;
  TRY(flags_status(ctx, ctx->h_flags[FLAGS_PASS1], "pass 1"));
  ctx->h_state = *ctx->h_state_pinned;
  return finish_solve(ctx, opts, fixed, mu, E_band, A_free);
}

int mag_solve_columns(mag_ctx* ctx, const mag_opts* opts, double* mu, double* E_band,
                      double* A_free) {
  TRY(ensure_system(ctx));
  TRY(check_opts(ctx, opts));
  const bool fixed = !std::isnan(opts->mu_fixed);
  if (!fixed && !(opts->n_electrons > 0.0 && opts->n_electrons < 2.0 * (double)ctx->M))
    return fail(ctx, MAG_EBRACKET, "n_electrons must lie in (0, 2M)");
  ctx->solved = false;
  ctx->density_ready = false;
  ctx->pass2_pending = false;
  ctx->adj_kept = false;
  ctx->opts = *opts;
  if (opts->workflow == MAG_WORKFLOW_AUTO) {
    const double need = 8.0 * (double)ctx->nnz * opts->nu;
    const double held = ctx->P.p ? (double)ctx->P.bytes : 0.0;  // reusable
    if (held >= need) {
      ctx->opts.workflow = MAG_WORKFLOW_STORE;  // P is already there: no new memory
    } else {
      // store when P takes at most half of the device memory that is free
      // (or held by the P buffer it replaces)
      size_t free_b = 0, total_b = 0;
      if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
      const double limit = 0.5 * ((double)free_b + held);
      ctx->opts.workflow = need <= limit ? MAG_WORKFLOW_STORE : MAG_WORKFLOW_RECOMPUTE;
    }
  }
  ctx->stats.workflow_used = ctx->opts.workflow;
  const int nu = opts->nu;
  ctx->nu = nu;
  const int64_t M = ctx->M;
  ALLOC(ctx->eps, sizeof(double) * M * nu);
  ALLOC(ctx->w, sizeof(double) * M * nu);
  ALLOC(ctx->nu_eff, sizeof(int32_t) * M);
  const bool store = ctx->opts.workflow == MAG_WORKFLOW_STORE;
  if (store) ALLOC(ctx->P, sizeof(double) * ctx->nnz * nu);
  if (opts->schedule == MAG_SCHED_GRAPH && graph_usable(ctx, ctx->opts))
    return replay_solve(ctx, opts, fixed, mu, E_band, A_free);

  // ---- pass 1, then mu and the energies, with one synchronisation at the end
  TRY(span_mark(ctx, SPAN_PASS1, 0));
  ColumnJob job;
  job.cols_dev = ctx->k_cols.as<int32_t>();
  job.cols_host = ctx->h_order;
  job.order = true;
  job.nu = nu;
  job.breakdown = opts->breakdown > 0 ? opts->breakdown : 1e-12;
  job.eig_sweeps = opts->eig_sweeps;
  job.schedule = opts->schedule;
  job.eps = ctx->eps.as<double>();
  job.w = ctx->w.as<double>();
  job.nu_eff = ctx->nu_eff.as<int32_t>();
  job.want_P = store ? 1 : 0;
  job.P_store = store ? ctx->P.as<double>() : nullptr;
  job.keep_adj = (opts->keep_exact && adjoint_supported(krylov_capacity(nu)) &&
                  opts->schedule != MAG_SCHED_GRAPH) ? 1 : 0;
  ctx->time_kernels = true;
  ctx->stats.t_krylov_ms = 0.0;
  ctx->stats.t_eig_ms = 0.0;
  ctx->stats.krylov_launches = 0;
  const int rc_pass1 = run_columns(ctx, job);
  ctx->time_kernels = false;
  TRY(rc_pass1);
  TRY(span_mark(ctx, SPAN_PASS1, 1));
  TRY(flags_enqueue(ctx, FLAGS_PASS1));
  // the mu kernels read only bounded ranges of the spectra, so they may run
  // before pass 1's flags are checked
  TRY(span_mark(ctx, SPAN_MU, 0));
  TRY(enqueue_mu(ctx, opts, fixed));
  HIPCHK(hipMemcpyAsync(ctx->h_state_pinned, ctx->state.p, sizeof(MuState),
                        hipMemcpyDeviceToHost, ctx->stream));
  TRY(span_mark(ctx, SPAN_MU, 1));
  TRY(sync(ctx));
  TRY(read_kernel_times(ctx));
  ctx->stats.t_pass1_ms = span_ms(ctx, SPAN_PASS1);
  ctx->stats.t_mu_ms = span_ms(ctx, SPAN_MU);
  TRY(flags_status(ctx, ctx->h_flags[FLAGS_PASS1], "pass 1"));
  ctx->h_state = *ctx->h_state_pinned;
  TRY(finish_solve(ctx, opts, fixed, mu, E_band, A_free));
  if (opts->schedule == MAG_SCHED_GRAPH) {
    const int rc = capture_solve(ctx, job, opts, fixed);
    if (rc != MAG_OK) return rc;
  }
  return MAG_OK;
}

int mag_spectra(mag_ctx* ctx, double* eps, double* w, int32_t* nu_eff, int mem_kind) {
  TRY(ensure_system(ctx));
  TRY(check_mem_kind(ctx, mem_kind));
  if (!ctx->solved) return fail(ctx, MAG_ESTATE, "no solve");
  TRY(copy_out(ctx, eps, ctx->eps.p, sizeof(double) * ctx->M * ctx->nu, mem_kind));
  TRY(copy_out(ctx, w, ctx->w.p, sizeof(double) * ctx->M * ctx->nu, mem_kind));
  TRY(copy_out(ctx, nu_eff, ctx->nu_eff.p, sizeof(int32_t) * ctx->M, mem_kind));
  return sync(ctx);
}

int mag_energy(mag_ctx* ctx, double* E_band, double* A_free, double* N_check, double* S_ent) {
  TRY(ensure_system(ctx));
  if (!ctx->solved) return fail(ctx, MAG_ESTATE, "no solve");
  if (E_band) *E_band = ctx->h_state.E;
  if (A_free) *A_free = ctx->h_state.E - ctx->opts.kT * ctx->h_state.S_ent;
  if (N_check) *N_check = ctx->h_state.N;
  if (S_ent) *S_ent = ctx->h_state.S_ent;
  return MAG_OK;
}

static int upload_cols(mag_ctx* ctx, const int32_t* cols, int64_t n, int mem_kind,
                       std::vector<int32_t>& host) {
  host.resize(n);
  if (n == 0) return MAG_OK;
  HIPCHK(hipMemcpyAsync(host.data(), cols, sizeof(int32_t) * n,
                        mem_kind == MAG_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost,
                        ctx->stream));
  TRY(sync(ctx));
  for (int32_t c : host)
    if (c < 0 || c >= ctx->M) return fail(ctx, MAG_EINVAL, "column id out of range");
  return MAG_OK;
}

int mag_column_spectra(mag_ctx* ctx, const mag_opts* opts, const int32_t* cols, int64_t n,
                       double* eps, double* w, int32_t* nu_eff, int mem_kind) {
  TRY(ensure_system(ctx));
  TRY(check_mem_kind(ctx, mem_kind));
  TRY(check_opts(ctx, opts));
  if (n < 0 || (n > 0 && !cols)) return fail(ctx, MAG_EINVAL, "bad column list");
  if (n == 0) return MAG_OK;
  ColumnJob job;
  TRY(upload_cols(ctx, cols, n, mem_kind, job.cols_host));
  DevBuf dcols, out;
  TRY(copy_in(ctx, dcols, job.cols_host.data(), sizeof(int32_t) * n, MAG_HOST));
  ALLOC(out, sizeof(double) * 2 * n * opts->nu + sizeof(int32_t) * n);
  job.cols_dev = dcols.as<int32_t>();
  job.nu = opts->nu;
  job.breakdown = opts->breakdown > 0 ? opts->breakdown : 1e-12;
  job.eig_sweeps = opts->eig_sweeps;
  job.schedule = opts->schedule;
  job.eps = out.as<double>();
  job.w = job.eps + n * opts->nu;
  job.nu_eff = reinterpret_cast<int32_t*>(job.w + n * opts->nu);
  job.out_by_slot = 1;
  TRY(run_columns(ctx, job));
  TRY(take_errors(ctx, "mag_column_spectra"));
  TRY(copy_out(ctx, eps, job.eps, sizeof(double) * n * opts->nu, mem_kind));
  TRY(copy_out(ctx, w, job.w, sizeof(double) * n * opts->nu, mem_kind));
  TRY(copy_out(ctx, nu_eff, job.nu_eff, sizeof(int32_t) * n, mem_kind));
  return sync(ctx);
}

// ---------------------------------------------------------------------------
// pass 2
// ---------------------------------------------------------------------------
int mag_density_matrix(mag_ctx* ctx, double* rho_csr, double* pi_csr, int mem_kind) {
  TRY(ensure_system(ctx));
  TRY(check_mem_kind(ctx, mem_kind));
  TRY(ensure_density(ctx));
  TRY(copy_out(ctx, rho_csr, ctx->rho.p, sizeof(double) * ctx->nnz, mem_kind));
  TRY(copy_out(ctx, pi_csr, ctx->pi.p, sizeof(double) * ctx->nnz, mem_kind));
  return sync(ctx);
}

// Krylov pass over selected columns writing every cluster row, then a
// per-chunk consumer (2: rho on the whole cluster column, 3: G(z) columns)
static int full_columns(mag_ctx* ctx, const mag_opts* o, const std::vector<int32_t>& hcols,
                        int consumer, const double* zdev, int nz, double* out_dev,
                        std::vector<int64_t>& off) {
  const int64_t n = (int64_t)hcols.size();
  const int64_t per = consumer == 3 ? 2 * (int64_t)nz : 1;
  std::vector<int64_t> soff(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) soff[i + 1] = soff[i] + NORB * ctx->h_clus_size[hcols[i] >> 2];
  off = soff;
  for (auto& x : soff) x *= (consumer == 3 ? (int64_t)nz : 1);  // complex-pair index base
  DevBuf dcols, spec, doff;
  TRY(copy_in(ctx, dcols, hcols.data(), sizeof(int32_t) * n, MAG_HOST));
  TRY(copy_in(ctx, doff, soff.data(), sizeof(int64_t) * (n + 1), MAG_HOST));
  ALLOC(spec, sizeof(double) * 2 * n * o->nu + sizeof(int32_t) * n);
  (void)per;
  ColumnJob job;
  job.cols_dev = dcols.as<int32_t>();
  job.cols_host = hcols;
  job.nu = o->nu;
  job.breakdown = o->breakdown > 0 ? o->breakdown : 1e-12;
  job.eig_sweeps = o->eig_sweeps;
  job.schedule = MAG_SCHED_GRID;
  job.full = 1;
  job.eps = spec.as<double>();
  job.w = job.eps + n * o->nu;
  job.nu_eff = reinterpret_cast<int32_t*>(job.w + n * o->nu);
  job.out_by_slot = 1;
  job.want_P = 1;
  job.consumer = consumer;
  job.out_off = doff.as<int64_t>();
  job.out = out_dev;
  job.z = zdev;
  job.nz = nz;
  TRY(run_columns(ctx, job));
  return take_errors(ctx, "cluster columns");
}

int mag_cluster_columns(mag_ctx* ctx, const int32_t* cols, int64_t n, double* rho_out,
                        int64_t* offsets, int mem_kind) {
  TRY(ensure_system(ctx));
  TRY(check_mem_kind(ctx, mem_kind));
  if (!ctx->solved) return fail(ctx, MAG_ESTATE, "no solve");
  if (n < 0 || (n > 0 && !cols)) return fail(ctx, MAG_EINVAL, "bad column list");
  std::vector<int32_t> hcols;
  TRY(upload_cols(ctx, cols, n, mem_kind, hcols));
  std::vector<int64_t> off(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + NORB * ctx->h_clus_size[hcols[i] >> 2];
  if (offsets) std::copy(off.begin(), off.end(), offsets);
  if (!rho_out || n == 0) return MAG_OK;
  DevBuf out;
  double* dst = rho_out;
  if (mem_kind == MAG_HOST) {
    ALLOC(out, sizeof(double) * std::max<int64_t>(off[n], 1));
    dst = out.as<double>();
  }
  std::vector<int64_t> o2;
  TRY(full_columns(ctx, &ctx->opts, hcols, 2, nullptr, 0, dst, o2));
  if (mem_kind == MAG_HOST) TRY(copy_out(ctx, rho_out, dst, sizeof(double) * off[n], MAG_HOST));
  return sync(ctx);
}

int mag_green_columns(mag_ctx* ctx, const mag_opts* opts, const int32_t* cols, int64_t n,
                      const double* z, int nz, double* G_out, int64_t* offsets, int mem_kind) {
  TRY(ensure_system(ctx));
  TRY(check_mem_kind(ctx, mem_kind));
  TRY(check_opts(ctx, opts));
  if (n < 0 || (n > 0 && !cols) || nz < 0 || (nz > 0 && !z))
    return fail(ctx, MAG_EINVAL, "bad column or energy list");
  std::vector<int32_t> hcols;
  TRY(upload_cols(ctx, cols, n, mem_kind, hcols));
  std::vector<int64_t> off(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + NORB * ctx->h_clus_size[hcols[i] >> 2];
  if (offsets) std::copy(off.begin(), off.end(), offsets);
  if (!G_out || n == 0 || nz == 0) return MAG_OK;
  DevBuf dz, out;
  TRY(copy_in(ctx, dz, z, sizeof(double) * 2 * nz, MAG_HOST));
  double* dst = G_out;
  if (mem_kind == MAG_HOST) {
    ALLOC(out, sizeof(double) * 2 * std::max<int64_t>(off[n] * nz, 1));
    dst = out.as<double>();
  }
  std::vector<int64_t> o2;
  TRY(full_columns(ctx, opts, hcols, 3, dz.as<double>(), nz, dst, o2));
  if (mem_kind == MAG_HOST)
    TRY(copy_out(ctx, G_out, dst, sizeof(double) * 2 * off[n] * nz, MAG_HOST));
  return sync(ctx);
}

int mag_cocg_columns(mag_ctx* ctx, const int32_t* cols, int64_t n, const double* z, int nz,
                     double tol, int max_iter, double* G_out, int64_t* offsets, int32_t* iters,
                     int mem_kind) {
  TRY(ensure_system(ctx));
  TRY(check_mem_kind(ctx, mem_kind));
  if (n < 0 || (n > 0 && !cols) || nz < 0 || (nz > 0 && !z))
    return fail(ctx, MAG_EINVAL, "bad column or energy list");
  if (!(tol > 0.0) || !std::isfinite(tol) || max_iter < 1)
    return fail(ctx, MAG_EINVAL, "need tol > 0 and max_iter >= 1");
  for (int q = 0; q < nz; ++q)
    if (!std::isfinite(z[2 * q]) || !std::isfinite(z[2 * q + 1]) || z[2 * q + 1] == 0.0)
      return fail(ctx, MAG_EINVAL, "energies must be finite with a nonzero imaginary part");
  std::vector<int32_t> hcols;
  TRY(upload_cols(ctx, cols, n, mem_kind, hcols));
  std::vector<int64_t> off(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + NORB * ctx->h_clus_size[hcols[i] >> 2];
  if (offsets) std::copy(off.begin(), off.end(), offsets);
  if (!G_out || n == 0 || nz == 0) return MAG_OK;
  Timer tm(ctx->stream);
  DevBuf dcols, dz, doff, out, dit;
  TRY(copy_in(ctx, dcols, hcols.data(), sizeof(int32_t) * n, MAG_HOST));
  TRY(copy_in(ctx, dz, z, sizeof(double) * 2 * nz, MAG_HOST));
  TRY(copy_in(ctx, doff, off.data(), sizeof(int64_t) * (n + 1), MAG_HOST));
  double* dst = G_out;
  if (mem_kind == MAG_HOST) {
    ALLOC(out, sizeof(double) * 2 * std::max<int64_t>(off[n] * nz, 1));
    dst = out.as<double>();
  }
  int32_t* pit = (mem_kind == MAG_DEVICE) ? iters : nullptr;
  if (!pit) {
    ALLOC(dit, sizeof(int32_t) * n * nz);
    pit = dit.as<int32_t>();
  }
  CocgArgs ca{};
  ca.cols = dcols.as<int32_t>();
  ca.ncols = n;
  ca.clus_ptr = ctx->clus_ptr.as<int64_t>();
  ca.clus_atoms = ctx->clus_atoms.as<int32_t>();
  ca.bptr = ctx->bptr.as<int32_t>();
  ca.bcol = ctx->bcol.as<int32_t>();
  ca.bval = ctx->bval.as<double>();
  ca.z = dz.as<double>();
  ca.nz = nz;
  ca.tol = tol;
  ca.max_iter = max_iter;
  ca.off = doff.as<int64_t>();
  ca.G = dst;
  ca.iters = pit;
  ca.err = ctx->errflag.as<int32_t>();
  for (int q0 = 0; q0 < nz; q0 += COCG_NZ) {
    ca.q0 = q0;
    HIPCHK(launch_cocg(ca, ctx->stream));
  }
  TRY(take_errors(ctx, "mag_cocg_columns"));
  ctx->stats.t_cocg_ms = tm.stop_ms();
  if (mem_kind == MAG_HOST)
    TRY(copy_out(ctx, G_out, dst, sizeof(double) * 2 * off[n] * nz, MAG_HOST));
  if (iters && mem_kind == MAG_HOST)
    TRY(copy_out(ctx, iters, pit, sizeof(int32_t) * n * nz, MAG_HOST));
  return sync(ctx);
}

// ---------------------------------------------------------------------------
// derivatives
// ---------------------------------------------------------------------------
int mag_backward(mag_ctx* ctx, double gA, double* dAdH_csr, double* dAdS_csr, int mem_kind) {
  TRY(ensure_system(ctx));
  TRY(check_mem_kind(ctx, mem_kind));
  if (!std::isfinite(gA)) return fail(ctx, MAG_EINVAL, "gA must be finite");
  TRY(ensure_density(ctx, true));
  DevBuf tmp;
  if (mem_kind == MAG_HOST && (dAdH_csr || dAdS_csr))
    ALLOC(tmp, sizeof(double) * 2 * ctx->nnz);
  if (dAdH_csr) {
    double* dst = mem_kind == MAG_HOST ? tmp.as<double>() : dAdH_csr;
    HIPCHK(launch_scale_copy(ctx->rho.as<double>(), ctx->nnz, gA, dst, ctx->stream));
    if (mem_kind == MAG_HOST) TRY(copy_out(ctx, dAdH_csr, dst, sizeof(double) * ctx->nnz, MAG_HOST));
  }
  if (dAdS_csr) {
    double* dst = mem_kind == MAG_HOST ? tmp.as<double>() + ctx->nnz : dAdS_csr;
    HIPCHK(launch_scale_copy(ctx->pi.as<double>(), ctx->nnz, -gA, dst, ctx->stream));
    if (mem_kind == MAG_HOST) TRY(copy_out(ctx, dAdS_csr, dst, sizeof(double) * ctx->nnz, MAG_HOST));
  }
  return settle(ctx, nullptr);
}

// the forces through rho and pi (pass 2 first if needed), enqueued only:
// the caller synchronises with settle()
static int forces_enqueue(mag_ctx* ctx, const mag_sk_model* model, double* F, int mem_kind,
                          DevBuf& out) {
  TRY(ensure_density(ctx, true));
  TRY(span_mark(ctx, SPAN_FORCES, 0));
  ALLOC(ctx->f_grad, sizeof(double) * 3 * ctx->N);
  ALLOC(ctx->f_part, sizeof(double) * 3 * std::max<int64_t>(ctx->nblk, 1));
  DevBuf& grad = ctx->f_grad;
  HIPCHK(launch_sk_vjp(to_dev(*model), ctx->pos.as<double>(), ctx->N, ctx->nblk, ctx->cell,
                       ctx->bptr.as<int32_t>(), ctx->bcol.as<int32_t>(),
                       ctx->btrans.as<int32_t>(), ctx->rho.as<double>(), ctx->pi.as<double>(),
                       -1.0, ctx->f_part.as<double>(), grad.as<double>(), ctx->stream));
  double* dst = F;
  if (mem_kind == MAG_HOST) {
    ALLOC(out, sizeof(double) * 3 * ctx->N);
    dst = out.as<double>();
  }
  HIPCHK(launch_scale_copy(grad.as<double>(), 3 * ctx->N, -1.0, dst, ctx->stream));
  if (mem_kind == MAG_HOST) TRY(copy_out(ctx, F, dst, sizeof(double) * 3 * ctx->N, MAG_HOST));
  TRY(span_mark(ctx, SPAN_FORCES, 1));
  return flags_enqueue(ctx, FLAGS_CALL);
}

int mag_forces(mag_ctx* ctx, const mag_sk_model* model, double* F, int mem_kind) {
  TRY(ensure_system(ctx));
  TRY(check_mem_kind(ctx, mem_kind));
  if (!model_ok(model)) return fail(ctx, MAG_EINVAL, "invalid Slater-Koster model");
  if (!F) return fail(ctx, MAG_EINVAL, "F is NULL");
  if (!ctx->has_pos) return fail(ctx, MAG_EINVAL, "forces need mag_system.pos");
  DevBuf out;  // host staging, alive until the synchronisation
  TRY(forces_enqueue(ctx, model, F, mem_kind, out));
  TRY(settle(ctx, "mag_forces"));
  ctx->stats.t_forces_ms = span_ms(ctx, SPAN_FORCES);
  return MAG_OK;
}

int mag_forces_exact(mag_ctx* ctx, const mag_sk_model* model, double* F, int mem_kind) {
  TRY(ensure_system(ctx));
  TRY(check_mem_kind(ctx, mem_kind));
  if (!model_ok(model)) return fail(ctx, MAG_EINVAL, "invalid Slater-Koster model");
  if (!F) return fail(ctx, MAG_EINVAL, "F is NULL");
  if (!ctx->has_pos) return fail(ctx, MAG_EINVAL, "forces need mag_system.pos");
  if (!ctx->solved) return fail(ctx, MAG_ESTATE, "no solve: call mag_solve_columns first");
  const int cap = krylov_capacity(ctx->nu);
  if (!adjoint_supported(cap))
    return fail(ctx, MAG_EUNSUPPORTED, "the exact gradient supports nu <= 30");
  if (adjoint_occupancy(cap) < 1)
    return fail(ctx, MAG_EUNSUPPORTED, "the exact-gradient kernel does not fit on this device");
  TRY(span_mark(ctx, SPAN_EXACT, 0));
  ALLOC(ctx->adj_fJ, sizeof(double) * 3 * std::max<int64_t>(ctx->clus_total, 1));
  ALLOC(ctx->adj_F, sizeof(double) * 3 * ctx->N);
  ColumnJob job;
  job.cols_dev = ctx->k_cols.as<int32_t>();
  job.cols_host = ctx->h_order;
  job.order = true;
  job.nu = ctx->nu;
  job.breakdown = ctx->opts.breakdown > 0 ? ctx->opts.breakdown : 1e-12;
  job.eig_sweeps = ctx->opts.eig_sweeps;
  job.schedule = MAG_SCHED_PERSISTENT;
  // the first pass's spectra stay as they are: this pass writes scratch rows
  ALLOC(ctx->tmp_cols, sizeof(double) * 2 * ctx->M * ctx->nu + sizeof(int32_t) * ctx->M);
  job.eps = ctx->tmp_cols.as<double>();
  job.w = job.eps + ctx->M * ctx->nu;
  job.nu_eff = reinterpret_cast<int32_t*>(job.w + ctx->M * ctx->nu);
  job.consumer = 4;
  job.skm = to_dev(*model);
  const mag_stats keep = ctx->stats;  // the pass-1 timings stay the solve's
  if (ctx->adj_kept) {
    // the solve kept every column's pass-1 data: no second pass
    TRY(adjoint_tail(ctx, job, ctx->k_cols.as<int32_t>(), ctx->adj_nu.as<int32_t>(), ctx->M, cap,
                     device_count_cus(ctx->device)));
  } else {
    TRY(run_columns(ctx, job));
  }
  ctx->stats.t_krylov_ms = keep.t_krylov_ms;
  ctx->stats.t_eig_ms = keep.t_eig_ms;
  ctx->stats.krylov_launches = keep.krylov_launches;
  ctx->stats.schedule_used = keep.schedule_used;
  ctx->stats.krylov_buckets = keep.krylov_buckets;
  ctx->stats.krylov_tpb = keep.krylov_tpb;
  ctx->stats.krylov_cache_blocks = keep.krylov_cache_blocks;
  HIPCHK(launch_gather_forces(ctx->clus_ptr.as<int64_t>(), ctx->clus_atoms.as<int32_t>(), ctx->N,
                              ctx->adj_fJ.as<double>(), ctx->adj_F.as<double>(), ctx->stream));
  TRY(copy_out(ctx, F, ctx->adj_F.p, sizeof(double) * 3 * ctx->N, mem_kind));
  TRY(span_mark(ctx, SPAN_EXACT, 1));
  TRY(flags_enqueue(ctx, FLAGS_CALL));
  TRY(settle(ctx, "mag_forces_exact"));
  ctx->stats.t_forces_exact_ms = span_ms(ctx, SPAN_EXACT);
  return MAG_OK;
}

int mag_icohp(mag_ctx* ctx, const mag_sk_model* model, double* B, double* B_sigma,
              double* B_pi, int mem_kind) {
  TRY(ensure_system(ctx));
  TRY(check_mem_kind(ctx, mem_kind));
  if (!model_ok(model)) return fail(ctx, MAG_EINVAL, "invalid Slater-Koster model");
  if (!B && !B_sigma && !B_pi) return fail(ctx, MAG_EINVAL, "no output requested");
  if (!ctx->has_pos) return fail(ctx, MAG_EINVAL, "ICOHP needs mag_system.pos");
  TRY(ensure_density(ctx));
  const int64_t nblk = ctx->nnz / 16;
  double* dst[3] = {B, B_sigma, B_pi};
  DevBuf out;
  if (mem_kind == MAG_HOST) {
    ALLOC(out, sizeof(double) * 3 * std::max<int64_t>(nblk, 1));
    for (int q = 0; q < 3; ++q)
      if (dst[q]) dst[q] = out.as<double>() + q * nblk;
  }
  Timer tm(ctx->stream);
  HIPCHK(launch_icohp(to_dev(*model), ctx->pos.as<double>(), ctx->N, nblk, ctx->cell,
                      ctx->bptr.as<int32_t>(), ctx->bcol.as<int32_t>(), ctx->bval.as<double>(),
                      ctx->rho.as<double>(), dst[0], dst[1], dst[2], ctx->stream));
  if (mem_kind == MAG_HOST) {
    double* host[3] = {B, B_sigma, B_pi};
    for (int q = 0; q < 3; ++q)
      if (host[q]) TRY(copy_out(ctx, host[q], dst[q], sizeof(double) * nblk, MAG_HOST));
  }
  TRY(sync(ctx));
  ctx->stats.t_icohp_ms = tm.stop_ms();
  return take_errors(ctx, "mag_icohp");
}

int mag_cohp(mag_ctx* ctx, const double* energies, int ne, double eta, double* C, int mem_kind) {
  TRY(ensure_system(ctx));
  TRY(check_mem_kind(ctx, mem_kind));
  if (!energies || !C || ne <= 0) return fail(ctx, MAG_EINVAL, "energies, ne > 0 and C required");
  if (!(eta >= 1e-100) || !std::isfinite(eta))
    return fail(ctx, MAG_EINVAL, "eta must be finite and >= 1e-100");
  for (int q = 0; q < ne; ++q)
    if (!std::isfinite(energies[q])) return fail(ctx, MAG_EINVAL, "energies must be finite");
  if (!ctx->solved) return fail(ctx, MAG_ESTATE, "no solve: call mag_solve_columns first");
  if (ctx->opts.workflow != MAG_WORKFLOW_STORE || !ctx->P.p)
    return fail(ctx, MAG_ESTATE, "COHP needs the stored pattern rows: solve with MAG_WORKFLOW_STORE");
  const int64_t nblk = ctx->nnz / 16;
  DevBuf en, out;
  ALLOC(en, sizeof(double) * ne);
  HIPCHK(hipMemcpyAsync(en.p, energies, sizeof(double) * ne, hipMemcpyHostToDevice, ctx->stream));
  double* dst = C;
  if (mem_kind == MAG_HOST) {
    ALLOC(out, sizeof(double) * std::max<int64_t>(1, nblk * ne));
    dst = out.as<double>();
  }
  Timer tm(ctx->stream);
  HIPCHK(launch_cohp(ctx->bval.as<double>(), ctx->bptr.as<int32_t>(), ctx->N, nblk,
                     ctx->rowptr.as<int64_t>(), ctx->P.as<double>(), ctx->eps.as<double>(),
                     ctx->nu_eff.as<int32_t>(), ctx->nu, en.as<double>(), ne, eta, dst,
                     ctx->stream));
  if (mem_kind == MAG_HOST) TRY(copy_out(ctx, C, dst, sizeof(double) * nblk * ne, MAG_HOST));
  TRY(sync(ctx));
  ctx->stats.t_cohp_ms = tm.stop_ms();
  return take_errors(ctx, "mag_cohp");
}

// E_rep (device scalar in md_sum[0]), e_atom (md_e) and F_rep (md_Frep) on
// the last build's pattern
static int pair_terms(mag_ctx* ctx, double phi0, double m_rep) {
  const int64_t n = ctx->sk_n;
  ALLOC(ctx->md_e, sizeof(double) * n);
  ALLOC(ctx->md_Frep, sizeof(double) * 3 * n);
  ALLOC(ctx->md_sum, sizeof(double) * 2);
  HIPCHK(launch_pair_rep(ctx->sk_model, ctx->sk_pos.as<double>(), n, ctx->sk_cell,
                         ctx->sk_bptr.as<int32_t>(), ctx->sk_bcol.as<int32_t>(), phi0, m_rep,
                         ctx->md_e.as<double>(), ctx->md_Frep.as<double>(), ctx->stream));
  HIPCHK(launch_sum(ctx->md_e.as<double>(), n, 0, ctx->md_sum.as<double>(), ctx->stream));
  return MAG_OK;
}

int mag_pair_repulsion(mag_ctx* ctx, double phi0, double m_rep, double* E_rep, double* e_atom,
                       double* F, int mem_kind) {
  if (!ctx) return MAG_EINVAL;
  TRY(check_mem_kind(ctx, mem_kind));
  if (!ctx->sk_built) return fail(ctx, MAG_ESTATE, "no Slater-Koster build");
  if (!std::isfinite(phi0) || !std::isfinite(m_rep) || !(m_rep > 0.0))
    return fail(ctx, MAG_EINVAL, "need finite phi0 and m_rep > 0");
  HIPCHK(hipSetDevice(ctx->device));
  TRY(pair_terms(ctx, phi0, m_rep));
  const int64_t n = ctx->sk_n;
  if (e_atom) TRY(copy_out(ctx, e_atom, ctx->md_e.p, sizeof(double) * n, mem_kind));
  if (F) TRY(copy_out(ctx, F, ctx->md_Frep.p, sizeof(double) * 3 * n, mem_kind));
  double e = 0.0;
  HIPCHK(hipMemcpyAsync(&e, ctx->md_sum.p, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  TRY(sync(ctx));
  if (E_rep) *E_rep = e;
  return MAG_OK;
}

// one frame of the MD run: build, system, solve, forces (into md_F) and the
// frame's energies; the kinetic energy is taken by the caller
static int md_frame(mag_ctx* ctx, const mag_sk_model* model, const mag_opts* opts,
                    const mag_md_opts* md, int64_t n, const double cell[3], double* th) {
  int64_t nnz = 0;
  TRY(mag_sk_build(ctx, model, n, ctx->md_x.as<double>(), cell, MAG_DEVICE, &nnz));
  mag_system sys{};
  sys.n_atoms = n;
  sys.nnz = nnz;
  sys.rowptr = ctx->sk_rowptr.as<int64_t>();
  sys.colind = ctx->sk_colind.as<int32_t>();
  sys.H = ctx->sk_H.as<double>();
  sys.S = ctx->sk_S.as<double>();
  sys.pos = ctx->md_x.as<double>();
  for (int d = 0; d < 3; ++d) sys.cell[d] = cell[d];
  sys.r_cluster = md->r_cluster;
  TRY(mag_set_system(ctx, &sys, MAG_DEVICE));
  double mu = 0.0, E = 0.0, A = 0.0;
  mag_opts fo = *opts;
  fo.keep_exact = md->exact_forces ? 1 : 0;  // the frame's exact gradient reuses pass 1
  TRY(mag_solve_columns(ctx, &fo, &mu, &E, &A));
  DevBuf unused;
  if (md->exact_forces)
    TRY(mag_forces_exact(ctx, model, ctx->md_F.as<double>(), MAG_DEVICE));
  else
    TRY(forces_enqueue(ctx, model, ctx->md_F.as<double>(), MAG_DEVICE, unused));
  // the pair term, then one synchronisation for the forces, the pair energy
  // and the flags of every kernel since the solve
  double* Erep = reinterpret_cast<double*>(ctx->h_flags + 8);
  *Erep = 0.0;
  if (md->phi0 != 0.0) {
    TRY(pair_terms(ctx, md->phi0, md->m_rep));
    HIPCHK(launch_axpy(ctx->md_F.as<double>(), ctx->md_Frep.as<double>(), 3 * n, 1.0,
                       ctx->stream));
    HIPCHK(hipMemcpyAsync(Erep, ctx->md_sum.p, sizeof(double), hipMemcpyDeviceToHost,
                          ctx->stream));
  }
  TRY(flags_enqueue(ctx, FLAGS_CALL));
  TRY(settle(ctx, "mag_md_run"));
  if (!md->exact_forces) ctx->stats.t_forces_ms = span_ms(ctx, SPAN_FORCES);
  th[0] = A + *Erep;
  th[2] = mu;
  th[3] = E;
  th[4] = *Erep;
  return MAG_OK;
}

static int md_kinetic(mag_ctx* ctx, const mag_md_opts* md, int64_t n, double* th) {
  ALLOC(ctx->md_sum, sizeof(double) * 2);
  HIPCHK(launch_sum(ctx->md_v.as<double>(), 3 * n, 1, ctx->md_sum.as<double>() + 1, ctx->stream));
  double vv = 0.0;
  HIPCHK(hipMemcpyAsync(&vv, ctx->md_sum.as<double>() + 1, sizeof(double), hipMemcpyDeviceToHost,
                        ctx->stream));
  TRY(sync(ctx));
  th[1] = 0.5 * md->mass * vv * AMU_A2_FS2_EV;
  return MAG_OK;
}

int mag_md_run(mag_ctx* ctx, const mag_sk_model* model, const mag_opts* opts,
               const mag_md_opts* md, int64_t n_atoms, const double cell[3], double* pos,
               double* vel, double* F, double* thermo, int mem_kind) {
  if (!ctx) return MAG_EINVAL;
  TRY(check_mem_kind(ctx, mem_kind));
  if (!model_ok(model)) return fail(ctx, MAG_EINVAL, "invalid Slater-Koster model");
  if (!opts || !md || !cell || !pos || !vel || !thermo)
    return fail(ctx, MAG_EINVAL, "NULL argument");
  if (n_atoms < 1) return fail(ctx, MAG_EINVAL, "need n_atoms >= 1");
  if (!(md->dt > 0.0) || !std::isfinite(md->dt) || !(md->mass > 0.0) ||
      !std::isfinite(md->mass) || md->n_steps < 0 || !std::isfinite(md->phi0) ||
      !std::isfinite(md->r_cluster) || (md->phi0 != 0.0 && !(md->m_rep > 0.0)) ||
      !std::isfinite(md->m_rep) || (md->exact_forces != 0 && md->exact_forces != 1))
    return fail(ctx, MAG_EINVAL,
                "need dt > 0, mass > 0, n_steps >= 0, finite phi0, m_rep > 0 and exact_forces "
                "0 or 1");
  HIPCHK(hipSetDevice(ctx->device));
  const int64_t n = n_atoms;
  ALLOC(ctx->md_x, sizeof(double) * 3 * n);
  ALLOC(ctx->md_v, sizeof(double) * 3 * n);
  ALLOC(ctx->md_F, sizeof(double) * 3 * n);
  HIPCHK(hipMemcpyAsync(ctx->md_x.p, pos, sizeof(double) * 3 * n, kind_in(mem_kind), ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->md_v.p, vel, sizeof(double) * 3 * n, kind_in(mem_kind), ctx->stream));
  HIPCHK(launch_check_finite(ctx->md_v.as<double>(), 3 * n, ctx->errflag.as<int32_t>(),
                             ctx->stream));
  TRY(take_errors(ctx, "mag_md_run"));
  // state back to the caller, also when a frame fails
  auto give_back = [&]() -> int {
    TRY(copy_out(ctx, pos, ctx->md_x.p, sizeof(double) * 3 * n, mem_kind));
    TRY(copy_out(ctx, vel, ctx->md_v.p, sizeof(double) * 3 * n, mem_kind));
    if (F) TRY(copy_out(ctx, F, ctx->md_F.p, sizeof(double) * 3 * n, mem_kind));
    return sync(ctx);
  };
  int rc = md_frame(ctx, model, opts, md, n, cell, thermo);
  if (rc == MAG_OK) rc = md_kinetic(ctx, md, n, thermo);
  if (rc != MAG_OK) {
    (void)give_back();
    return rc;
  }
  const double c = 0.5 * md->dt / (md->mass * AMU_A2_FS2_EV);
  const auto t0 = std::chrono::steady_clock::now();
  for (int step = 1; step <= md->n_steps; ++step) {
    double* th = thermo + 5 * (int64_t)step;
    rc = (launch_md_kick(ctx->md_v.as<double>(), ctx->md_F.as<double>(), 3 * n, c, ctx->stream) ==
          hipSuccess)
             ? MAG_OK
             : fail(ctx, MAG_EHIP, "MD kick launch failed");
    if (rc == MAG_OK &&
        launch_md_drift(ctx->md_x.as<double>(), ctx->md_v.as<double>(), n, md->dt, cell,
                        ctx->stream) != hipSuccess)
      rc = fail(ctx, MAG_EHIP, "MD drift launch failed");
    if (rc == MAG_OK) rc = md_frame(ctx, model, opts, md, n, cell, th);
    if (rc == MAG_OK &&
        launch_md_kick(ctx->md_v.as<double>(), ctx->md_F.as<double>(), 3 * n, c, ctx->stream) !=
            hipSuccess)
      rc = fail(ctx, MAG_EHIP, "MD kick launch failed");
    if (rc == MAG_OK) rc = md_kinetic(ctx, md, n, th);
    if (rc != MAG_OK) {
      (void)give_back();
      return rc;
    }
  }
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  ctx->stats.t_md_step_ms = md->n_steps > 0 ? ms / md->n_steps : 0.0;
  return give_back();
}

int mag_get_stats(mag_ctx* ctx, mag_stats* out) {
  if (!ctx || !out) return MAG_EINVAL;
  int64_t bytes = 0;
  const DevBuf* bufs[] = {&ctx->sk_pos, &ctx->sk_bptr, &ctx->sk_bcol, &ctx->sk_rowptr,
                          &ctx->sk_colind, &ctx->sk_H, &ctx->sk_S, &ctx->rowptr, &ctx->bptr,
                          &ctx->bcol, &ctx->btrans, &ctx->bval, &ctx->pos, &ctx->clus_ptr,
                          &ctx->clus_atoms, &ctx->eps, &ctx->w, &ctx->nu_eff, &ctx->state,
                          &ctx->partials, &ctx->P, &ctx->rho, &ctx->pi, &ctx->k_hs,
                          &ctx->k_urow, &ctx->k_qpat, &ctx->k_nu, &ctx->k_npat, &ctx->k_cols,
                          &ctx->k_queue, &ctx->errflag, &ctx->tmp_cols, &ctx->tmp_off,
                          &ctx->tmp_out, &ctx->k_trid, &ctx->k_evu, &ctx->k_rot,
                          &ctx->k_sweep, &ctx->k_qlst, &ctx->k_fbl, &ctx->k_fbc,
                          &ctx->md_x, &ctx->md_v, &ctx->md_F, &ctx->md_Frep, &ctx->md_e,
                          &ctx->md_sum, &ctx->f_part, &ctx->f_grad, &ctx->k_slots,
                          &ctx->k_qbeg, &ctx->adj_cvec, &ctx->adj_cdg, &ctx->adj_hbar,
                          &ctx->adj_wbar, &ctx->adj_fJ, &ctx->adj_F, &ctx->adj_counter,
                          &ctx->adj_q, &ctx->adj_r, &ctx->adj_h, &ctx->adj_beta, &ctx->adj_nu, &ctx->sk_cnt,
                          &ctx->sys_tmp, &ctx->sys_cnt, &ctx->sys_nz};
  for (const DevBuf* b : bufs) bytes += (int64_t)b->bytes;
  for (const CellList* c : {&ctx->sk_cells, &ctx->sys_cells})
    bytes += (int64_t)(c->cell_of.bytes + c->cell_count.bytes + c->cell_start.bytes +
                       c->cell_atoms.bytes);
  ctx->stats.device_bytes = bytes;
  *out = ctx->stats;
  return MAG_OK;
}

}  // extern "C"
