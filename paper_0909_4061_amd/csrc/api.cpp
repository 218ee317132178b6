// Host side of the C ABI declared in include/rsvd.h: argument validation,
// the workspace plan, the split-K choice, and the kernel sequences of the
// hot-path calls (range finder, power steps, projection, small SVD + lifts).
//
// The kernel sequence of one problem is written once, against a Runner: the
// single-problem calls launch each kernel at once on the caller's stream; the
// batched call records the sequence of every problem, turns each step into
// one launch over all problems (kernel families with a batched entry), and
// replays the recorded launches from a HIP graph cached on the handle.
//
// Every call enqueues its kernels on the caller's stream and returns without
// synchronizing.  Argument errors are found here, before any launch.
#include <algorithm>
#include <cstring>
#include <new>
#include <cmath>
#include <vector>

#include "common.hpp"

namespace {
struct BatchPlan;
}

struct rsvd_handle_s {
  int device;
  int32_t* status;  // device word: RSVD_FLAG_* bits accumulated by the kernels
  char* scratch = nullptr;  // device address of this device's copy of `scratch` (rsvd_full_static)
  // optional launch timing (rsvd_profile_enable)
  std::vector<hipEvent_t> events;  // 2 per record
  std::vector<int> kinds;          // family of each record
  int used = 0;
  uint32_t mask = ~0u;             // families that are timed
  // batched calls: recorded launch plans (device tables + graph), most recent last
  std::vector<BatchPlan*> plans;
  hipStream_t capture = nullptr;  // stream the batched graphs are captured on
};

// Workspace of rsvd_full_static, for callers that cannot allocate: one copy
// per device, held from the library's first use on that device until the
// process ends.  Host code never passes `scratch` itself to a kernel (its
// host-side name is not a device address): rsvd_create looks up the device
// address once, with the handle's device current, and every launch takes that.
static __device__ __align__(256) unsigned char scratch[RSVD_STATIC_SCRATCH_BYTES];

namespace {

using namespace rsvd;

constexpr size_t kAlign = 256;
constexpr size_t kMaxPlans = 8;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

struct Split {
  int32_t S;
  int64_t kchunk;
};

Split no_split(int64_t K) { return Split{1, std::max<int64_t>(K, 1)}; }

// Split the contraction range K so that (row blocks x S) workgroups cover the
// 256 CUs about twice, keeping at least four K stages per workgroup.
Split choose_split(int64_t rows, int64_t K, const GemmTile& t) {
  const int64_t nrb = std::max<int64_t>(1, ceil_div(rows, t.bm));
  int64_t S = ceil_div(512, nrb);
  const int64_t smax = std::max<int64_t>(1, K / (4 * (int64_t)t.bk));
  S = std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(S, smax), 16));
  const int64_t kchunk = round_up(ceil_div(K, S), t.bk);
  S = ceil_div(K, kchunk);
  return Split{(int32_t)S, kchunk};
}

struct Plan {
  int64_t m, n, l, k, Mx;
  int32_t Lp, Lg;
  int esize;
  int dtype, prec;
  bool stream;  // FP32 data: the A-streaming products take the streaming kernels (X packed first)
  Split nn, tn;
  size_t omega, part, Y, Qt, pack, gpart, G, R1, R2, R3, Rt, Rb, RinvT, XU, XV, Uh, sig, flags, srft_d,
      srft_R, eigV, eigZ, eigT, omega2, sx, eig2, gsrft_tab, gsrft_at, total;
};

bool valid_enum(int32_t v, int32_t lo, int32_t hi) { return v >= lo && v <= hi; }

rsvd_status validate(const rsvd_problem* pr) {
  if (!pr) return RSVD_E_INVAL;
  if (pr->m < 1 || pr->n < 1 || pr->k < 1 || pr->p < 0 || pr->q < 0) return RSVD_E_INVAL;
  if (pr->lda < pr->n) return RSVD_E_INVAL;
  if (!valid_enum(pr->dtype, RSVD_F32, RSVD_F64) || !valid_enum(pr->sketch, RSVD_GAUSSIAN, RSVD_GSRFT) ||
      !valid_enum(pr->prec, RSVD_NATIVE, RSVD_BF16X3))
    return RSVD_E_INVAL;
  const int64_t l = (int64_t)pr->k + pr->p;
  if (l > std::min(pr->m, pr->n)) return RSVD_E_INVAL;
  if (l > RSVD_MAX_L) return RSVD_E_UNSUPPORTED;
  if (pr->dtype == RSVD_F64 && pr->prec != RSVD_NATIVE) return RSVD_E_UNSUPPORTED;
  if (pr->sketch != RSVD_GAUSSIAN) {
    // One row of A, as n/2 complex values, is transformed in a workgroup's LDS.
    const int64_t nmax = int64_t{2} << (pr->dtype == RSVD_F64 ? SRFT_MAX_LOGN_F64 : SRFT_MAX_LOGN_F32);
    if (pr->q != 0 || pr->n < 8 || pr->n > nmax || (pr->n & (pr->n - 1)) != 0) return RSVD_E_UNSUPPORTED;
    // the Givens chains: a row and its gathered copy in LDS
    if (pr->sketch == RSVD_GSRFT && !gsrft_shape_ok(pr->dtype, pr->n)) return RSVD_E_UNSUPPORTED;
  }
  return RSVD_OK;
}

// The second eigensolver of the two-sided single pass (byte offsets in its
// region): G (Lg x Lg), reflectors V (l x EIG_LDV), Z (l x l), T (d, e, tau,
// the eigenvalues, the norm bound, the flags), Uh (l x l), sig (l), XU and XV
// (l x k elements), S (k elements).
struct Eig2Layout {
  size_t G, V, Z, T, Uh, sig, XU, XV, S, total;
};
Eig2Layout eig2_layout(const Plan& P) {
  Eig2Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += align_up(std::max<size_t>(bytes, 1));
    return at;
  };
  const size_t ll8 = (size_t)P.l * P.l * 8;
  L.G = take((size_t)P.Lg * P.Lg * 8);
  L.V = take((size_t)P.l * EIG_LDV * 8);
  L.Z = take(ll8);
  L.T = take((size_t)(4 * P.l + 1) * 8 + (size_t)P.l * 4);
  L.Uh = take(ll8);
  L.sig = take((size_t)P.l * 8);
  L.XU = take((size_t)P.l * P.k * P.esize);
  L.XV = take((size_t)P.l * P.k * P.esize);
  L.S = take((size_t)P.k * P.esize);
  L.total = off;
  return L;
}
size_t eig2_bytes(const Plan& P) { return eig2_layout(P).total; }

// Workspace regions of one problem.  `batched`: no split-K (every problem of
// a batch runs the same launch sequence, and the batch itself fills the chip);
// `stream`: the products with A take the streaming kernels.
Plan make_plan(const rsvd_problem* pr, bool batched = false, bool stream = true) {
  Plan P{};
  P.m = pr->m;
  P.n = pr->n;
  P.l = (int64_t)pr->k + pr->p;
  P.k = pr->k;
  P.Mx = std::max(P.m, P.n);
  P.dtype = pr->dtype;
  P.prec = pr->prec;
  P.esize = pr->dtype == RSVD_F64 ? 8 : 4;
  P.stream = stream && pr->dtype == RSVD_F32;
  const GemmTile big = gemm_tile(pr->dtype, pr->prec);
  // padded width of the A-streaming products' X and split-K partials (128 for
  // the BF16 streaming kernels, see gemm())
  P.Lp = (P.stream && pr->prec != RSVD_NATIVE) ? 128 : (int32_t)round_up(P.l, big.lp_mult);
  P.Lg = (int32_t)round_up(P.l, 16);
  // A batch of large matrices fills the chip without a split; a batch taking the
  // general GEMM splits K beyond 1024 so that its largest problems do not
  // leave one long workgroup per row block running after the rest.
  auto batch_split = [&](int64_t K) {
    if (stream || K <= 1024) return no_split(K);
    const int64_t kc = round_up(ceil_div(K, ceil_div(K, 1024)), big.bk);
    return Split{(int32_t)ceil_div(K, kc), kc};
  };
  P.nn = batched ? batch_split(P.n) : choose_split(P.m, P.n, big);
  P.tn = batched ? batch_split(P.m) : choose_split(P.n, P.m, big);
  int64_t part_elems = 0;
  if (P.nn.S > 1) part_elems = std::max(part_elems, (int64_t)P.nn.S * P.m * P.Lp);
  if (P.tn.S > 1) part_elems = std::max(part_elems, (int64_t)P.tn.S * P.n * P.Lp);
  const size_t es = (size_t)P.esize;
  const size_t ll8 = (size_t)P.l * P.l * 8;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += align_up(std::max<size_t>(bytes, 1));
    return at;
  };
  P.omega = take((size_t)P.n * P.l * es);
  P.part = take((size_t)part_elems * es);
  P.Y = take((size_t)P.Mx * P.l * es);
  P.Qt = take((size_t)P.n * P.l * es);
  P.pack = take(P.stream ? (size_t)stream_pack_bytes(P.Mx, 128) : 0);
  P.gpart = take((size_t)ceil_div(P.Mx, GRAM_ROWS) * P.Lg * P.Lg * 8);
  P.G = take((size_t)P.Lg * P.Lg * 8);
  P.R1 = take(ll8);
  P.R2 = take(ll8);
  P.R3 = take(ll8);
  P.Rt = take(ll8);
  P.Rb = take(ll8);
  P.RinvT = take((size_t)P.l * P.l * es);
  P.XU = take((size_t)P.l * P.k * es);
  P.XV = take((size_t)P.l * P.k * es);
  P.Uh = take(ll8);
  P.sig = take((size_t)P.l * 8);
  P.flags = take(64);
  P.srft_d = take(pr->sketch != RSVD_GAUSSIAN ? (size_t)P.n * 8 : 0);
  P.srft_R = take(pr->sketch != RSVD_GAUSSIAN ? (size_t)P.l * 4 : 0);
  // the Givens-chain sketch: its tables and the transformed copy of A
  P.gsrft_tab = take(pr->sketch == RSVD_GSRFT ? gsrft_table_bytes(P.n, P.esize) : 0);
  P.gsrft_at = take(pr->sketch == RSVD_GSRFT ? (size_t)P.m * P.n * es : 0);
  // eigensolver of the small SVD (FP32 data) and of the symmetric Stage B (a
  // single problem of either type): reflectors, eigenvectors, then d, e, tau,
  // the eigenvalues, the norm bound and the flags
  const bool eig = pr->dtype == RSVD_F32 || !batched;
  P.eigV = take(eig ? (size_t)P.l * EIG_LDV * 8 : 0);
  P.eigZ = take(eig ? ll8 : 0);
  P.eigT = take(eig ? (size_t)(4 * P.l + 1) * 8 + (size_t)P.l * 4 : 0);
  // the two-sided single pass (single problems): its second test matrix (m x l) and
  // four l x l FP64 matrices for the least-squares core
  P.omega2 = take(batched ? 0 : (size_t)P.m * P.l * es);
  P.sx = take(batched ? 0 : 4 * ll8);
  // and the eigensolver of its second Gram matrix, which runs beside the first
  P.eig2 = take(batched ? 0 : eig2_bytes(P));
  P.total = off;
  return P;
}

// Brackets one launch with a pair of events when timing is on.
struct Timed {
  rsvd_handle h;
  hipStream_t st;
  int idx = -1;
  Timed(rsvd_handle h_, int kind, hipStream_t st_) : h(h_), st(st_) {
    if (h && h->used < (int)h->kinds.size() && ((h->mask >> kind) & 1u)) {
      idx = h->used++;
      h->kinds[idx] = kind;
      (void)hipEventRecord(h->events[2 * idx], st);
    }
  }
  ~Timed() {
    if (idx >= 0) (void)hipEventRecord(h->events[2 * idx + 1], st);
  }
};

// ---------------------------------------------------------------------------
// Where the kernels of one problem go.
class Runner {
 public:
  virtual ~Runner() = default;
  virtual bool records() const = 0;
  virtual hipError_t gemm(int dtype, int prec, bool trans, const GemmParams& p, int kind) = 0;
  // the A-streaming product: X packed into p.pack, then the streaming kernel
  virtual hipError_t pack_x(int prec, const GemmParams& p) = 0;
  virtual hipError_t stream_gemm(int prec, bool trans, const GemmParams& p, int kind) = 0;
  virtual hipError_t gram_partial(int dtype, const GramParams& p) = 0;
  virtual hipError_t sum_parts(int dtype, const GramParams& p) = 0;
  virtual hipError_t gram_reduce(const GramReduceParams& p) = 0;
  virtual hipError_t chol(const CholParams& p) = 0;
  virtual hipError_t jacobi(const JacobiParams& p) = 0;
  virtual hipError_t eig(int stage, const EigParams& p) = 0;
  virtual hipError_t omega(int dtype, const OmegaParams& p) = 0;
  virtual hipError_t trmm(const TrmmParams& p) = 0;
  virtual hipError_t copy(const CopyParams& p) = 0;
  // adjoint pieces
  virtual hipError_t svd_adj_coef(const SvdAdjParams& p) = 0;
  virtual hipError_t qr_adj_sym(const QrSymParams& p) = 0;
  virtual hipError_t tri_inv(const TriInvParams& p) = 0;
  virtual hipError_t copy2d(const Copy2dParams& p) = 0;
};

// Launches at once on a stream (timed when the handle's timing is on).
class DirectRunner final : public Runner {
 public:
  DirectRunner(rsvd_handle h, hipStream_t st) : h_(h), st_(st) {}
  bool records() const override { return false; }
  hipError_t gemm(int dtype, int prec, bool trans, const GemmParams& p, int kind) override {
    Timed t(h_, kind, st_);
    return launch_gemm(dtype, prec, trans, p, st_);
  }
  hipError_t pack_x(int prec, const GemmParams& p) override {
    Timed t(h_, RSVD_KERNEL_PACK, st_);
    return launch_pack_x(prec, p, st_);
  }
  hipError_t stream_gemm(int prec, bool trans, const GemmParams& p, int kind) override {
    Timed t(h_, kind, st_);
    return launch_stream_gemm(prec, trans, p, st_);
  }
  hipError_t gram_partial(int dtype, const GramParams& p) override {
    Timed t(h_, RSVD_KERNEL_GRAM, st_);
    return launch_gram_partial(dtype, p, st_);
  }
  hipError_t sum_parts(int dtype, const GramParams& p) override {
    Timed t(h_, RSVD_KERNEL_GRAM, st_);
    return launch_sum_parts(dtype, p, st_);
  }
  hipError_t gram_reduce(const GramReduceParams& p) override {
    Timed t(h_, RSVD_KERNEL_GRAM, st_);
    return launch_gram_reduce(p.gpart, p.nblk, p.Lg, p.G, p.status, p.gate, st_);
  }
  hipError_t chol(const CholParams& p) override {
    Timed t(h_, RSVD_KERNEL_CHOL, st_);
    return launch_chol(p, st_);
  }
  hipError_t jacobi(const JacobiParams& p) override {
    Timed t(h_, RSVD_KERNEL_JACOBI, st_);
    return launch_jacobi(p, st_);
  }
  hipError_t eig(int stage, const EigParams& p) override {
    Timed t(h_, RSVD_KERNEL_EIG, st_);
    return launch_eig(stage, p, st_);
  }
  hipError_t omega(int dtype, const OmegaParams& p) override {
    return launch_omega(dtype, p.omega, p.n, p.l, p.seed, p.sid, st_);
  }
  hipError_t trmm(const TrmmParams& p) override { return launch_trmm_upper(p.R2, p.R1, p.R, p.l, p.gate, st_); }
  hipError_t copy(const CopyParams& p) override { return launch_copy_f64(p.src, p.dst, p.count, p.gate, st_); }
  hipError_t svd_adj_coef(const SvdAdjParams& p) override { return launch_svd_adj_coef(p, st_); }
  hipError_t qr_adj_sym(const QrSymParams& p) override { return launch_qr_adj_sym(p, st_); }
  hipError_t tri_inv(const TriInvParams& p) override { return launch_tri_inv_upper(p, st_); }
  hipError_t copy2d(const Copy2dParams& p) override { return launch_copy2d(p, st_); }

 private:
  rsvd_handle h_;
  hipStream_t st_;
};

// One step of a batched plan: the same kernel family and variant for every
// problem, with the problems' parameter blocks side by side.
enum SlotKind {
  SK_GEMM, SK_GRAM_PARTIAL, SK_GRAM_REDUCE, SK_CHOL, SK_JACOBI, SK_OMEGA, SK_TRMM, SK_COPY,
  SK_SUM_PARTS, SK_SVD_ADJ, SK_QR_SYM, SK_TRI_INV, SK_COPY2D, SK_PACK, SK_STREAM, SK_EIG
};

struct Slot {
  SlotKind kind;
  int dtype, prec;
  bool trans;
  size_t psize;
  std::vector<unsigned char> params;  // problem-major, psize bytes each
  std::vector<int64_t> blocks;        // workgroups of each problem
};

// Appends one problem's launches to the slots, in order; every problem of a
// batch must produce the same sequence of (family, variant).
class RecordRunner final : public Runner {
 public:
  explicit RecordRunner(std::vector<Slot>& slots) : slots_(slots) {}
  bool records() const override { return true; }
  size_t cursor() const { return cursor_; }
  hipError_t gemm(int dtype, int prec, bool trans, const GemmParams& p, int) override {
    return add(SK_GEMM, dtype, prec, trans, p, p.rows > 0 ? gemm_blocks(dtype, prec, p) : 0);
  }
  hipError_t pack_x(int prec, const GemmParams& p) override {
    if (!stream_params_ok(prec, p)) return hipErrorInvalidValue;
    return add(SK_PACK, 0, prec, false, p, p.rows > 0 ? pack_x_blocks(p) : 0);
  }
  hipError_t stream_gemm(int prec, bool trans, const GemmParams& p, int) override {
    if (!stream_params_ok(prec, p)) return hipErrorInvalidValue;
    return add(SK_STREAM, p.wide, prec, trans, p, stream_gemm_blocks(p));  // the dtype slot holds `wide`
  }
  hipError_t gram_partial(int dtype, const GramParams& p) override {
    return add(SK_GRAM_PARTIAL, dtype, 0, false, p, p.rows > 0 ? gram_partial_blocks(p) : 0);
  }
  hipError_t sum_parts(int dtype, const GramParams& p) override {
    if (p.rows > 0 && !sum_parts_ok(dtype, p)) return hipErrorInvalidValue;
    return add(SK_SUM_PARTS, dtype, 0, false, p, sum_parts_blocks(dtype, p));
  }
  hipError_t gram_reduce(const GramReduceParams& p) override {
    return add(SK_GRAM_REDUCE, 0, 0, false, p, gram_reduce_blocks(p));
  }
  hipError_t chol(const CholParams& p) override { return add(SK_CHOL, 0, 0, false, p, 1); }
  hipError_t jacobi(const JacobiParams& p) override { return add(SK_JACOBI, 0, jacobi_maxl_, false, p, 1); }
  int jacobi_maxl_ = 128;  // the Jacobi variant every problem of the batch runs
  // eigensolver stage s is recorded with the stage in the dtype slot and the
  // variant every problem of the batch runs in the prec slot
  hipError_t eig(int stage, const EigParams& p) override {
    return add(SK_EIG, stage, eig_maxl_, false, p, eig_blocks(stage, p));
  }
  int eig_maxl_ = 128;
  hipError_t omega(int dtype, const OmegaParams& p) override {
    return add(SK_OMEGA, dtype, 0, false, p, omega_blocks(p));
  }
  hipError_t trmm(const TrmmParams& p) override { return add(SK_TRMM, 0, 0, false, p, trmm_blocks(p)); }
  hipError_t copy(const CopyParams& p) override {
    return add(SK_COPY, 0, 0, false, p, p.count > 0 ? copy_blocks(p) : 0);
  }
  hipError_t svd_adj_coef(const SvdAdjParams& p) override {
    if (!svd_adj_coef_ok(p)) return hipErrorInvalidValue;
    return add(SK_SVD_ADJ, 0, 0, false, p, svd_adj_coef_blocks(p));
  }
  hipError_t qr_adj_sym(const QrSymParams& p) override {
    return add(SK_QR_SYM, 0, 0, false, p, qr_adj_sym_blocks(p));
  }
  hipError_t tri_inv(const TriInvParams& p) override {
    if (!tri_inv_ok(p)) return hipErrorInvalidValue;
    return add(SK_TRI_INV, 0, 0, false, p, 1);
  }
  hipError_t copy2d(const Copy2dParams& p) override { return add(SK_COPY2D, 0, 0, false, p, copy2d_blocks(p)); }

 private:
  template <typename P>
  hipError_t add(SlotKind kind, int dtype, int prec, bool trans, const P& p, int64_t blocks) {
    if (cursor_ == slots_.size()) slots_.push_back(Slot{kind, dtype, prec, trans, sizeof(P), {}, {}});
    Slot& s = slots_[cursor_++];
    if (s.kind != kind || s.dtype != dtype || s.prec != prec || s.trans != trans || s.psize != sizeof(P))
      return hipErrorInvalidValue;
    const auto* b = reinterpret_cast<const unsigned char*>(&p);
    s.params.insert(s.params.end(), b, b + sizeof(P));
    s.blocks.push_back(blocks);
    return hipSuccess;
  }
  std::vector<Slot>& slots_;
  size_t cursor_ = 0;
};

struct Ctx {
  const Plan& P;
  char* ws;
  hipStream_t st;   // for the launches only the single-problem path makes
  int32_t* status;
  rsvd_handle h;    // for timing; null when recording
  Runner* run;
  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(ws + off);
  }
  int32_t* shift_flag() const { return at<int32_t>(P.flags); }
};

#define RSVD_TRY(expr)                              \
  do {                                              \
    if ((expr) != hipSuccess) return RSVD_E_DEVICE; \
  } while (0)

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// op(A) X with the given arithmetic.  With `part` non-null and a split S > 1
// the result is left as partial products; otherwise it is written to `out`.
rsvd_status gemm(const Ctx& c, int prec, bool trans, const void* A, int64_t lda, int64_t rows, int64_t K,
                 const void* X, int64_t ldx, int32_t ncols, void* out, int64_t ldo, const Split& sp, void* part,
                 const int32_t* gate, bool streams_a = false, bool accum = false, void* pack = nullptr,
                 bool wide = false) {
  const GemmTile t = gemm_tile(c.P.dtype, prec);
  GemmParams g{};
  g.A = A;
  g.lda = lda;
  g.rows = rows;
  g.K = K;
  g.X = X;
  g.ldx = ldx;
  g.ncols = ncols;
  g.Lp = (int32_t)round_up(ncols, t.lp_mult);
  g.out = out;
  g.ldo = ldo;
  g.part = part;
  g.S = sp.S;
  g.kchunk = sp.kchunk;
  const int vec_mult = c.P.esize == 8 ? 2 : 4;
  g.vec = (lda % vec_mult == 0 && aligned16(A)) ? 1 : 0;
  g.gate = gate;
  g.accum = accum ? 1 : 0;
  g.narrow = (!c.run->records() && !streams_a && c.P.dtype == RSVD_F32 && prec == RSVD_NATIVE) ? 1 : 0;
  if (g.S > 1 && !part) return RSVD_E_INVAL;
  if (accum && (g.S > 1 || streams_a)) return RSVD_E_INVAL;
  const int kind = streams_a ? (trans ? RSVD_KERNEL_STREAM_TN : RSVD_KERNEL_STREAM_NN) : RSVD_KERNEL_SMALL_GEMM;
  if (streams_a && c.P.stream) {
    // BF16 products pad X to 128 columns: the streaming kernel's branch-free
    // steady-state loop needs all four 32-column tiles, and these products are
    // bound by HBM, not by the padded MFMA work.  FP32 products are bound by
    // the MFMA rate and keep the 32-column rounding.
    g.wide = wide && prec != RSVD_NATIVE ? 1 : 0;
    g.Lp = prec == RSVD_NATIVE ? (int32_t)round_up(ncols, 32) : (int32_t)round_up(std::max(ncols, 128), 128);
    if (g.S > 1 && g.Lp != c.P.Lp) return RSVD_E_INVAL;  // partials are read with the plan's width
    g.pack = pack ? pack : c.at<void>(c.P.pack);
    RSVD_TRY(c.run->pack_x(prec, g));
    RSVD_TRY(c.run->stream_gemm(prec, trans, g, kind));
  } else {
    RSVD_TRY(c.run->gemm(c.P.dtype, prec, trans, g, kind));
  }
  return RSVD_OK;
}

// Gram of a rows x l matrix into G (FP64, Lg x Lg upper).  Source: split-K
// partials (summed and stored into `y` first) or a stored `y`.
rsvd_status gram(const Ctx& c, bool from_part, const Split& sp, void* y, int64_t rows, const int32_t* gate) {
  GramParams g{};
  g.part = c.at<void>(c.P.part);
  g.S = sp.S;
  g.Lp = c.P.Lp;
  g.yin = y;
  g.yout = y;
  g.ldy = c.P.l;
  g.rows = rows;
  g.l = (int32_t)c.P.l;
  g.Lg = c.P.Lg;
  g.gpart = c.at<double>(c.P.gpart);
  g.gate = gate;
  const int64_t nchunks = gram_geometry(rows, c.P.Lg, !c.run->records(), &g.tgroups, &g.chunk);
  if (from_part || c.run->records()) {  // a recorded problem without a split takes the (empty) step
    GramParams gs = g;
    if (!from_part) gs.rows = 0;
    RSVD_TRY(c.run->sum_parts(c.P.dtype, gs));
  }
  RSVD_TRY(c.run->gram_partial(c.P.dtype, g));
  const GramReduceParams r{g.gpart, nchunks, c.P.Lg, c.at<double>(c.P.G), c.status, gate};
  RSVD_TRY(c.run->gram_reduce(r));
  return RSVD_OK;
}

rsvd_status chol(const Ctx& c, int64_t rows, double* R, bool want_inv, const int32_t* gate, int32_t* shifted,
                 bool reset_shifted = false) {
  CholParams q{};
  q.G = c.at<double>(c.P.G);
  q.Lg = c.P.Lg;
  q.l = (int32_t)c.P.l;
  q.rows = rows;
  q.R = R;
  q.Rinv = nullptr;  // only R^-1 in the element type (RinvT) is used downstream
  q.RinvT = want_inv ? c.at<void>(c.P.RinvT) : nullptr;
  q.dtype = c.P.dtype;
  q.shifted = shifted;
  q.reset_shifted = reset_shifted ? 1 : 0;
  q.status = c.status;
  q.gate = gate;
  RSVD_TRY(c.run->chol(q));
  return RSVD_OK;
}

// CholeskyQR2 (plus a third pass when a shift was needed) of a rows x l matrix.
// Source: the split-K partials of the GEMM that produced it (from_part; the sum
// is stored into `y`) or `y` itself.  Q (rows x l) may alias y.  If R_out is
// non-null it receives the combined triangular factor.
//
// full == false (the bases inside the power scheme that only feed the next
// product): the second pass, like the third, runs only when the first needed a
// shift.  One pass with the FP64 Gram leaves Q = fl(Y R^-1) orthonormal to
// about u kappa(Y) (u of the element type): a well-conditioned basis of the
// same range, which is all the next application of A or A* uses, and no more
// accurate a range than Y stored in the element type carries anyway.  A
// shifted first pass (Y numerically rank deficient) takes all three passes, as
// the final basis does.
rsvd_status orth(const Ctx& c, bool from_part, const Split& sp, void* y, int64_t rows, void* Q, double* R_out,
                 bool full = true) {
  const int64_t l = c.P.l;
  int32_t* flag = c.shift_flag();  // cleared by the first factorization, set by a shifted one
  double* Rs[3] = {c.at<double>(c.P.R1), c.at<double>(c.P.R2), c.at<double>(c.P.R3)};
  for (int pass = 0; pass < 3; ++pass) {
    const int32_t* gate = (pass == 2 || (pass == 1 && !full)) ? flag : nullptr;
    const bool src_part = pass == 0 && from_part;
    void* src = pass == 0 ? y : Q;
    rsvd_status s = gram(c, src_part, sp, src, rows, gate);
    if (s != RSVD_OK) return s;
    // R itself only when the combined factor is wanted: R^-1 (rounded to the
    // element type) is all the apply step reads
    s = chol(c, rows, R_out ? Rs[pass] : nullptr, true, gate, pass < 2 ? flag : nullptr, pass == 0);
    if (s != RSVD_OK) return s;
    s = gemm(c, RSVD_NATIVE, false, src, l, rows, l, c.at<void>(c.P.RinvT), l, (int32_t)l, Q, l, no_split(l),
             nullptr, gate);
    if (s != RSVD_OK) return s;
  }
  if (R_out) {
    // R = R3 R2 R1 (R3 only when the shifted third pass ran)
    RSVD_TRY(c.run->trmm(TrmmParams{Rs[1], Rs[0], R_out, (int32_t)l, nullptr}));
    RSVD_TRY(c.run->trmm(TrmmParams{Rs[2], R_out, c.at<double>(c.P.Rt), (int32_t)l, flag}));
    RSVD_TRY(c.run->copy(CopyParams{c.at<double>(c.P.Rt), R_out, l * l, flag}));
  }
  return RSVD_OK;
}

// Y = A X (NN, rows m) or A^T X (TN, rows n), orthonormalized into Q (one
// CholeskyQR pass unless `full` or a shift, see orth).
rsvd_status apply_and_orth(const Ctx& c, const rsvd_problem* pr, bool trans, const void* A, const void* X,
                           void* Q, bool full) {
  const Plan& P = c.P;
  const Split& sp = trans ? P.tn : P.nn;
  const int64_t rows = trans ? P.n : P.m;
  const int64_t K = trans ? P.m : P.n;
  void* y = c.at<void>(P.Y);
  rsvd_status s = gemm(c, pr->prec, trans, A, pr->lda, rows, K, X, P.l, (int32_t)P.l, y, P.l, sp,
                       sp.S > 1 ? c.at<void>(P.part) : nullptr, nullptr, true);
  if (s != RSVD_OK) return s;
  return orth(c, sp.S > 1, sp, y, rows, Q, nullptr, full);
}

// Sum the S split-K partial products (rows x l) into `out` in a fixed order.
rsvd_status reduce_parts(const Ctx& c, const Split& sp, int64_t rows, void* out) {
  if (sp.S == 1 && !c.run->records()) return RSVD_OK;
  if (sp.S == 1) rows = 0;  // a recorded problem without a split takes the (empty) step
  GramParams g{};
  g.part = c.at<void>(c.P.part);
  g.S = sp.S;
  g.Lp = c.P.Lp;
  g.yout = out;
  g.ldy = c.P.l;
  g.rows = rows;
  g.l = (int32_t)c.P.l;
  RSVD_TRY(c.run->sum_parts(c.P.dtype, g));
  return RSVD_OK;
}

// Y = A Omega (m x l) for either test matrix, into `y` (left as split-K
// partials for the Gaussian GEMM when the plan splits it).
rsvd_status sketch(const Ctx& c, const rsvd_problem* pr, const void* A, void* y) {
  const Plan& P = c.P;
  if (pr->sketch != RSVD_GAUSSIAN) {
    if (c.run->records()) return RSVD_E_UNSUPPORTED;
    const void* src = A;
    int64_t ld = pr->lda;
    if (pr->sketch == RSVD_GSRFT) {
      // A D'' Theta' D' Theta into the workspace copy, which the SRFT then sketches
      void* tab = c.at<void>(P.gsrft_tab);
      void* at = c.at<void>(P.gsrft_at);
      RSVD_TRY(launch_gsrft_draw(pr->dtype, tab, pr->n, pr->seed, pr->stream_id, c.st));
      {
        Timed t_(c.h, RSVD_KERNEL_GSRFT, c.st);
        RSVD_TRY(launch_gsrft_rows(pr->dtype, A, pr->lda, pr->m, pr->n, tab, at, c.st));
      }
      src = at;
      ld = pr->n;
    }
    double* d = c.at<double>(P.srft_d);
    int32_t* R = c.at<int32_t>(P.srft_R);
    RSVD_TRY(launch_srft_draw(d, R, pr->n, (int32_t)P.l, pr->seed, pr->stream_id, c.st));
    Timed t_(c.h, RSVD_KERNEL_SRFT, c.st);
    RSVD_TRY(launch_srft_rows(pr->dtype, src, ld, pr->m, pr->n, (int32_t)P.l, d, R, y, c.st));
    return RSVD_OK;
  }
  void* omega = c.at<void>(P.omega);
  RSVD_TRY(c.run->omega(pr->dtype, OmegaParams{omega, pr->n, (int32_t)P.l, pr->seed, pr->stream_id}));
  return gemm(c, pr->prec, false, A, pr->lda, P.m, P.n, omega, P.l, (int32_t)P.l, y, P.l, P.nn,
              P.nn.S > 1 ? c.at<void>(P.part) : nullptr, nullptr, true);
}

// --- the steps of the hot path, shared by the single and batched calls -----

// Algorithm 4.1 steps 2-3 / Algorithm 4.5: Q = orth(A Omega).
// full == false (problem->q > 0: power steps follow): the basis only feeds the
// first power step, so it takes one CholeskyQR pass like the other inner bases
// (see orth).
rsvd_status range_finder_steps(const Ctx& c, const rsvd_problem* pr, const void* A, void* Q, bool full = true) {
  void* y = c.at<void>(c.P.Y);
  const bool parts = pr->sketch == RSVD_GAUSSIAN && c.P.nn.S > 1;
  rsvd_status s = sketch(c, pr, A, y);
  if (s != RSVD_OK) return s;
  return orth(c, parts, c.P.nn, y, pr->m, Q, nullptr, full);
}

// Algorithm 4.4 steps 3-6.
rsvd_status power_steps(const Ctx& c, const rsvd_problem* pr, const void* A, void* Q) {
  void* Qt = c.at<void>(c.P.Qt);
  for (int j = 0; j < pr->q; ++j) {
    // every basis but the last only feeds the next product: one CholeskyQR pass
    rsvd_status s = apply_and_orth(c, pr, true, A, Q, Qt, false);  // Qt = orth(A^T Q)
    if (s != RSVD_OK) return s;
    s = apply_and_orth(c, pr, false, A, Qt, Q, j == pr->q - 1);  // Q = orth(A Qt)
    if (s != RSVD_OK) return s;
  }
  return RSVD_OK;
}

// Algorithm 5.1 step 1: Bt = A^T Q.
rsvd_status project_steps(const Ctx& c, const rsvd_problem* pr, const void* A, const void* Q, void* Bt) {
  const Plan& P = c.P;
  const Split& sp = P.tn;
  rsvd_status s = gemm(c, pr->prec, true, A, pr->lda, P.n, P.m, Q, P.l, (int32_t)P.l, Bt, P.l, sp,
                       sp.S > 1 ? c.at<void>(P.part) : nullptr, nullptr, true);
  if (s != RSVD_OK) return s;
  return reduce_parts(c, sp, P.n, Bt);
}

// Algorithm 5.1 steps 2-3 and truncation: the SVD of the small matrix B gives
// U~ and Sigma, and V = B* U~ Sigma^-1.  For FP64 data through a triangular
// factor R of B* from CholeskyQR2 (a shifted third pass when needed) and
// one-sided Jacobi on C = R^T (C C^T = B B*), which is backward stable:
// singular values carry absolute errors of order u sigma_1.  For FP32 data
// from the FP64 Gram B B*, whose error (u_64 sigma_1^2 / sigma_j relative to
// sigma_j) stays below what FP32 arithmetic resolves.
rsvd_status small_svd(const Ctx& c, const void* Bt, void* S, JacobiParams& j) {
  const Plan& P = c.P;
  double* R = c.at<double>(P.R1);
  rsvd_status s;
  j = JacobiParams{};
  j.R = R;
  j.l = (int32_t)P.l;
  j.k = (int32_t)P.k;
  j.dtype = P.dtype;
  j.Uh = c.at<double>(P.Uh);
  j.sig = c.at<double>(P.sig);
  j.XU = c.at<void>(P.XU);
  j.XV = c.at<void>(P.XV);
  j.S = S;
  j.status = c.status;
  if (P.dtype == RSVD_F64) {
    R = c.at<double>(P.Rb);
    j.R = R;
    // Q_B (n x l) goes to the Y region, unused by now; Bt itself is only read.
    s = orth(c, false, no_split(1), const_cast<void*>(Bt), P.n, c.at<void>(P.Y), R);
    if (s != RSVD_OK) return s;
    RSVD_TRY(c.run->jacobi(j));
    return RSVD_OK;
  }
  // FP32 data: from the FP64 Gram B B*.  A single problem takes its
  // eigendecomposition B B* = U~ S^2 U~* (tridiagonalization, then one wave per
  // eigenpair over many CUs); a batch, whose problems already fill the chip one
  // workgroup each, takes one-sided Jacobi on C = R^T with R^T R = B B*
  // (Cholesky), the same Gram accuracy in fewer workgroups.
  s = gram(c, false, no_split(1), const_cast<void*>(Bt), P.n, nullptr);
  if (s != RSVD_OK) return s;
  if (c.run->records()) {
    s = chol(c, P.n, R, false, nullptr, nullptr);
    if (s != RSVD_OK) return s;
    RSVD_TRY(c.run->jacobi(j));
    return RSVD_OK;
  }
  EigParams e{};
  e.G = c.at<double>(P.G);
  e.Lg = P.Lg;
  e.l = (int32_t)P.l;
  e.k = (int32_t)P.k;
  e.dtype = P.dtype;
  e.V = c.at<double>(P.eigV);
  e.Z = c.at<double>(P.eigZ);
  double* t = c.at<double>(P.eigT);
  e.tri = t;
  e.lam = t + 3 * P.l;
  e.tnorm = t + 4 * P.l;
  e.flag = reinterpret_cast<int32_t*>(t + 4 * P.l + 1);
  e.Uh = j.Uh;
  e.sig = j.sig;
  e.XU = j.XU;
  e.XV = j.XV;
  e.S = S;
  e.status = c.status;
  for (int stage = 0; stage < 3; ++stage) RSVD_TRY(c.run->eig(stage, e));
  return RSVD_OK;
}

rsvd_status svd_steps(const Ctx& c, const void* Bt, const void* Q, void* U, void* S, void* V) {
  const Plan& P = c.P;
  JacobiParams j;
  rsvd_status s = small_svd(c, Bt, S, j);
  if (s != RSVD_OK) return s;
  // U = Q U~_k (m x k), V = Bt U~_k S_k^-1 (n x k)
  s = gemm(c, RSVD_NATIVE, false, Q, P.l, P.m, P.l, j.XU, P.k, (int32_t)P.k, U, P.k, no_split(P.l), nullptr,
           nullptr);
  if (s != RSVD_OK) return s;
  return gemm(c, RSVD_NATIVE, false, Bt, P.l, P.n, P.l, j.XV, P.k, (int32_t)P.k, V, P.k, no_split(P.l), nullptr,
              nullptr);
}

// ---------------------------------------------------------------------------
// Adjoint of the fixed-Omega randomized SVD: (gU, gS, gV) -> gA.

// Workspace of the adjoint, after the forward plan: every basis of the forward
// (Q_0..Q_q, Qt_1..Qt_q) with its combined triangular factor, B*, the
// adjoint temporaries, and the two factors of gA = Left RightT.
struct BwdLayout {
  Plan P;
  int q;
  int64_t Kc;         // (2q + 2) l
  int64_t gA_chunks;  // 128-column launches of gA = Left RightT (a batch pads to its widest problem)
  size_t Qs, Qts, Rs, Rts, Bt, gBt, gQ, gQt, gYt, T1, T2, Mq, Z, W1, M1p64, UhT, Rinv, Sy, W64, SW64, M2_64, Ukt64,
      M1p, W, SW, M2, Ukt, Sk, Left, RightT, part, gApack, total;
};

constexpr int64_t kBwdMaxSplit = 16;  // K chunks of the adjoint's transposed products

BwdLayout bwd_layout(const rsvd_problem* pr, bool batched = false, bool stream = true) {
  BwdLayout L{};
  L.P = make_plan(pr, batched, stream);
  const Plan& P = L.P;
  L.q = pr->q;
  L.Kc = (int64_t)(2 * pr->q + 2) * P.l;
  L.gA_chunks = ceil_div(P.n, 128);
  const size_t es = (size_t)P.esize, ml = (size_t)(P.m * P.l) * es, nl = (size_t)(P.n * P.l) * es;
  const size_t ll8 = (size_t)(P.l * P.l) * 8, lle = (size_t)(P.l * P.l) * es;
  const size_t lk8 = (size_t)(P.l * P.k) * 8, lke = (size_t)(P.l * P.k) * es;
  size_t off = P.total;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += align_up(std::max<size_t>(bytes, 1));
    return at;
  };
  L.Qs = take(ml * (size_t)(L.q + 1));
  L.Qts = take(nl * (size_t)std::max(L.q, 1));
  L.Rs = take(ll8 * (size_t)(L.q + 1));
  L.Rts = take(ll8 * (size_t)std::max(L.q, 1));
  L.Bt = take(nl);
  L.gBt = take(nl);
  L.gQ = take(ml);
  L.gQt = take(nl);
  L.gYt = take(nl);
  L.T1 = take(lke);
  L.T2 = take(lke);
  L.Mq = take(lle);
  L.Z = take(ll8);
  L.W1 = take(ll8);
  L.M1p64 = take(ll8);
  L.UhT = take(ll8);
  L.Rinv = take(ll8);
  L.Sy = take(ll8);
  L.W64 = take(ll8);
  L.SW64 = take(ll8);
  L.M2_64 = take(lk8);
  L.Ukt64 = take(lk8);
  L.M1p = take(lle);
  L.W = take(lle);
  L.SW = take(lle);
  L.M2 = take(lke);
  L.Ukt = take(lke);
  L.Sk = take((size_t)P.k * es);
  L.Left = take((size_t)(P.m * L.Kc) * es);
  L.RightT = take((size_t)(L.Kc * P.n) * es);
  L.part = take((size_t)kBwdMaxSplit * P.l * 128 * es);  // split-K partials, rows <= l, Lp <= 128
  // packed RightT for the streaming launches of gA: K = Kc rows, all columns at
  // once (BF16 products) or 128 per launch (FP32)
  const int32_t gA_lp = P.prec != RSVD_NATIVE ? (int32_t)round_up(P.n, 128) : 128;
  L.gApack = take(P.stream ? (size_t)stream_pack_bytes(L.Kc, gA_lp) : 0);
  L.total = off;
  return L;
}

rsvd_status copy2d(const Ctx& c, const void* src, int sdt, int64_t lds, void* dst, int ddt, int64_t ldd, int64_t rows,
                   int64_t cols, bool trans, bool negate = false) {
  const Copy2dParams p{src, sdt, lds, dst, ddt, ldd, rows, cols, trans ? 1 : 0, negate ? 1 : 0};
  RSVD_TRY(c.run->copy2d(p));
  return RSVD_OK;
}

// out (rows x ncols, ldo) = A^T X for the adjoint's products with few output rows
// (rows <= l) and a long contraction K: the K range is split over up to
// kBwdMaxSplit workgroups and the partial products summed in a fixed order.
rsvd_status gemm_tn_splitk_into(const Ctx& c, void* part_buf, const void* A, int64_t lda, int64_t rows, int64_t K,
                                const void* X, int64_t ldx, int32_t ncols, void* out, int64_t ldo) {
  const GemmTile t = gemm_tile(c.P.dtype, RSVD_NATIVE);
  Split sp = choose_split(rows, K, t);
  if (sp.S > kBwdMaxSplit) sp = Split{(int32_t)kBwdMaxSplit, round_up(ceil_div(K, kBwdMaxSplit), t.bk)};
  void* part = sp.S > 1 ? part_buf : nullptr;
  rsvd_status s = gemm(c, RSVD_NATIVE, true, A, lda, rows, K, X, ldx, ncols, out, ldo, sp, part, nullptr);
  if (s != RSVD_OK) return s;
  GramParams g{};
  g.part = part;
  g.S = sp.S;
  g.Lp = (int32_t)round_up(ncols, t.lp_mult);
  g.yout = out;
  g.ldy = ldo;
  g.rows = sp.S > 1 ? rows : 0;  // a recorded problem without a split still takes the (empty) step
  g.l = ncols;
  if (sp.S > 1 || c.run->records()) RSVD_TRY(c.run->sum_parts(c.P.dtype, g));
  return RSVD_OK;
}

// C = X1^T X2 (c1 x c2) over n rows with exact FP64 products (cross kernel, the
// plan's Gram partial region): into out (element type) or, sym, its symmetric
// part into the plan's G.
hipError_t cross(const Ctx& c, const void* X1, int64_t ld1, const void* X2, int64_t ld2, int64_t rows, int32_t c1,
                 int32_t c2, void* out, int64_t ldo, bool sym, bool out_f64 = false) {
  Timed t_(c.h, RSVD_KERNEL_GRAM, c.st);
  const CrossParams x{X1, ld1, X2, ld2, rows, c1, c2, c.P.dtype, c.P.Lg, c.at<double>(c.P.gpart),
                      cross_blocks(rows), sym ? 1 : 0, out, ldo, c.at<double>(c.P.G), out_f64 ? 1 : 0};
  return launch_cross(x, c.st);
}

// The eigensolver of an l x l symmetric matrix held in G (FP64 upper triangle):
// tridiagonalization, eigenpairs, cluster fix-up.  Outputs in the plan's Uh,
// sig, XU, XV (value order, the first k); S (k, element type) is scratch here.
EigParams eig_params(const Ctx& c, void* S) {
  const Plan& P = c.P;
  EigParams e{};
  e.G = c.at<double>(P.G);
  e.Lg = P.Lg;
  e.l = (int32_t)P.l;
  e.k = (int32_t)P.k;
  e.dtype = P.dtype;
  e.V = c.at<double>(P.eigV);
  e.Z = c.at<double>(P.eigZ);
  double* t = c.at<double>(P.eigT);
  e.tri = t;
  e.lam = t + 3 * P.l;
  e.tnorm = t + 4 * P.l;
  e.flag = reinterpret_cast<int32_t*>(t + 4 * P.l + 1);
  e.Uh = c.at<double>(P.Uh);
  e.sig = c.at<double>(P.sig);
  e.XU = c.at<void>(P.XU);
  e.XV = c.at<void>(P.XV);
  e.S = S;
  e.status = c.status;
  return e;
}

// Algorithm 5.3 (nystrom == false) and Algorithm 5.5 (nystrom == true) for a
// symmetric / psd n x n A and a basis Q (n x l).  Single problems only.
rsvd_status herm_steps(const Ctx& c, const rsvd_problem* pr, const void* A, const void* Q, void* U, void* Lam,
                       bool nystrom) {
  const Plan& P = c.P;
  if (c.run->records()) return RSVD_E_UNSUPPORTED;
  const int64_t n = P.n, l = P.l;
  void* y = c.at<void>(P.Y);
  // B1 = A Q (n x l): the one pass over A
  rsvd_status s = gemm(c, pr->prec, false, A, pr->lda, n, n, Q, l, (int32_t)l, y, l, P.nn,
                       P.nn.S > 1 ? c.at<void>(P.part) : nullptr, nullptr, true);
  if (s != RSVD_OK) return s;
  s = reduce_parts(c, P.nn, n, y);
  if (s != RSVD_OK) return s;
  // the symmetric part of B = Q^T B1 (l x l) into G: exact FP64 products summed over chunks of rows
  RSVD_TRY(cross(c, Q, l, y, l, n, (int32_t)l, (int32_t)l, nullptr, 0, true));
  EigParams e = eig_params(c, Lam);
  EigPickParams pick{e.lam, e.Uh, e.sig, (int32_t)l, (int32_t)P.k, nystrom ? 0 : 1, P.dtype, Lam, nullptr};
  if (!nystrom) {
    // B = V Lambda V^T; the k of largest |lambda| and their vectors; U = Q V_k
    for (int stage = 0; stage < 3; ++stage) RSVD_TRY(c.run->eig(stage, e));
    pick.XU = c.at<void>(P.XU);
    {
      Timed t_(c.h, RSVD_KERNEL_EIG, c.st);
      RSVD_TRY(launch_eig_pick(pick, c.st));
    }
    return gemm(c, RSVD_NATIVE, false, Q, l, n, l, pick.XU, P.k, (int32_t)P.k, U, P.k, no_split(l), nullptr,
                nullptr);
  }
  // B2 = C^T C (C = R, upper; shifted when B2 is not positive definite to working
  // precision), F = B1 C^-1 in place of B1
  s = chol(c, n, nullptr, true, nullptr, c.shift_flag(), true);
  if (s != RSVD_OK) return s;
  s = gemm(c, RSVD_NATIVE, false, y, l, n, l, c.at<void>(P.RinvT), l, (int32_t)l, y, l, no_split(l), nullptr,
           nullptr);
  if (s != RSVD_OK) return s;
  // F = U Sigma V^T from the FP64 Gram F^T F = V Sigma^2 V^T: U = F V Sigma^-1 (XV), Lam = Sigma^2
  s = gram(c, false, no_split(1), y, n, nullptr);
  if (s != RSVD_OK) return s;
  for (int stage = 0; stage < 3; ++stage) RSVD_TRY(c.run->eig(stage, e));
  {
    Timed t_(c.h, RSVD_KERNEL_EIG, c.st);
    RSVD_TRY(launch_eig_pick(pick, c.st));
  }
  return gemm(c, RSVD_NATIVE, false, y, l, n, l, c.at<void>(P.XV), P.k, (int32_t)P.k, U, P.k, no_split(l), nullptr,
              nullptr);
}

// A plan for k columns over the same workspace regions (each sized for l >= k).
Plan narrowed_plan(const Plan& P, int64_t cols) {
  Plan q = P;
  q.l = cols;
  q.Lg = (int32_t)round_up(cols, 16);
  return q;
}

// Algorithm 5.6 (eigenvalue decomposition of a symmetric A in one pass over it)
// with the oversampled basis of the closing remark of Section 5.5.
rsvd_status onepass_steps(const Ctx& c, const rsvd_problem* pr, const void* A, void* U, void* Lam) {
  const Plan& P = c.P;
  if (c.run->records() || pr->sketch != RSVD_GAUSSIAN) return RSVD_E_UNSUPPORTED;
  const int64_t n = P.n, l = P.l, k = P.k;
  const Plan Pk = narrowed_plan(P, k);
  const Ctx ck{Pk, c.ws, c.st, c.status, c.h, c.run};
  // Y = A Omega (the one pass; Omega drawn into the plan's omega region)
  void* Y = c.at<void>(P.Qt);
  void* Q = c.at<void>(P.Y);
  rsvd_status s = sketch(c, pr, A, Y);
  if (s == RSVD_OK) s = reduce_parts(c, P.nn, n, Y);
  if (s != RSVD_OK) return s;
  if (k == l) {
    // no oversampling: Q = an orthonormal basis of range(Y) (CholeskyQR2)
    s = orth(c, false, no_split(1), Y, n, Q, nullptr);
  } else {
    // Q = the k leading left singular vectors of Y: Y = W S V^T from the small SVD of Y^T
    // (as for B^T in Algorithm 5.1), Q = Y V_k S_k^-1, then CholeskyQR2 of Q
    JacobiParams j;
    s = small_svd(c, Y, Lam, j);
    if (s == RSVD_OK)
      s = gemm(c, RSVD_NATIVE, false, Y, l, n, l, j.XV, k, (int32_t)k, Q, k, no_split(l), nullptr, nullptr);
    if (s == RSVD_OK) s = orth(ck, false, no_split(1), Q, n, Q, nullptr);
  }
  if (s != RSVD_OK) return s;
  // M = Q^T Omega, N = Q^T Y (k x l)
  void* M = c.at<void>(P.XU);
  void* N = c.at<void>(P.Rb);
  void* Mt = c.at<void>(P.XV);
  if (cross(c, Q, k, c.at<void>(P.omega), l, n, (int32_t)k, (int32_t)l, M, l, false) != hipSuccess ||
      cross(c, Q, k, Y, l, n, (int32_t)k, (int32_t)l, N, l, false) != hipSuccess)
    return RSVD_E_DEVICE;
  // least squares B M = N with M of full row rank: M^T = Q_M R_M (CholeskyQR2, l x k),
  // B = N Q_M R_M^-T; then its symmetric part
  if (s == RSVD_OK) s = copy2d(c, M, P.dtype, l, Mt, P.dtype, k, k, l, true);
  double* Rm = c.at<double>(P.Uh);
  if (s == RSVD_OK) s = orth(ck, false, no_split(1), Mt, l, Mt, Rm);
  if (s != RSVD_OK) return s;
  double* Rmi = c.at<double>(P.eigZ);
  RSVD_TRY(c.run->tri_inv(TriInvParams{Rm, Rmi, (int32_t)k}));
  void* RmiT = c.at<void>(P.R1);
  s = copy2d(c, Rmi, RSVD_F64, k, RmiT, P.dtype, k, k, k, true);
  void* T1 = c.at<void>(P.R2);
  void* Bu = c.at<void>(P.R3);
  if (s == RSVD_OK)
    s = gemm(c, RSVD_NATIVE, false, N, l, k, l, Mt, k, (int32_t)k, T1, k, no_split(l), nullptr, nullptr);
  if (s == RSVD_OK)
    s = gemm(c, RSVD_NATIVE, false, T1, k, k, k, RmiT, k, (int32_t)k, Bu, k, no_split(k), nullptr, nullptr);
  if (s != RSVD_OK) return s;
  {
    Timed t_(c.h, RSVD_KERNEL_EIG, c.st);
    RSVD_TRY(launch_sym_gram(SymGramParams{Bu, P.dtype, (int32_t)k, (int32_t)k, Pk.Lg, c.at<double>(P.G)}, c.st));
  }
  // B = V Lambda V^T (k x k), every pair kept in decreasing |lambda|; U = Q V
  EigParams e = eig_params(ck, Lam);
  for (int stage = 0; stage < 3; ++stage) RSVD_TRY(c.run->eig(stage, e));
  EigPickParams pick{e.lam, e.Uh, e.sig, (int32_t)k, (int32_t)k, 1, P.dtype, Lam, c.at<void>(P.XU)};
  {
    Timed t_(c.h, RSVD_KERNEL_EIG, c.st);
    RSVD_TRY(launch_eig_pick(pick, c.st));
  }
  return gemm(ck, RSVD_NATIVE, false, Q, k, n, k, pick.XU, k, (int32_t)k, U, k, no_split(k), nullptr, nullptr);
}

// The two-sided single pass for a general A (Section 5.5): Y = A Omega and
// Yt = A^T Omegat, Q = orth(Y), Qt = orth(Yt) (CholeskyQR2, so Q^T Y = R and
// Qt^T Yt = Rt), B (l x l) the minimum-residual solution of B M1 = R and
// B^T M2 = Rt with M1 = Qt^T Omega, M2 = Q^T Omegat: the normal equations
// B G1 + G2 B = R M1^T + M2 Rt^T (G1 = M1 M1^T, G2 = M2 M2^T), solved through
// the eigendecompositions of G1 and G2; then the SVD of B (its FP64 Gram and
// the eigensolver), U = Q Ub_k, V = Qt B^T Ub_k S_k^-1.
rsvd_status svd_onepass_steps(const Ctx& c, const rsvd_problem* pr, const void* A, void* U, void* S, void* V) {
  const Plan& P = c.P;
  if (c.run->records() || pr->sketch != RSVD_GAUSSIAN) return RSVD_E_UNSUPPORTED;
  const int64_t m = P.m, n = P.n, l = P.l, k = P.k;
  const int32_t li = (int32_t)l;
  const Plan p64 = [&] {
    Plan q = P;
    q.dtype = RSVD_F64;
    q.esize = 8;
    return q;
  }();
  const Ctx c64{p64, c.ws, c.st, c.status, c.h, c.run};
  double* X[4];
  for (int i = 0; i < 4; ++i) X[i] = c.at<double>(P.sx) + (int64_t)i * l * l;
  double* R1 = c.at<double>(P.R1);
  double* R2 = c.at<double>(P.R2);
  double* R3 = c.at<double>(P.R3);
  double* Rt = c.at<double>(P.Rt);
  double* G = c.at<double>(P.G);
  const int64_t Lg = P.Lg;
  void* Y = c.at<void>(P.Y);       // m x l, then Q
  void* Yt = c.at<void>(P.Qt);     // n x l, then Qt
  void* Om2 = c.at<void>(P.omega2);
  // the one pass: Y = A Omega, Yt = A^T Omegat (Omegat from (seed, stream_id with its top bit flipped))
  rsvd_status s = sketch(c, pr, A, Y);
  if (s == RSVD_OK) s = reduce_parts(c, P.nn, m, Y);
  if (s != RSVD_OK) return s;
  RSVD_TRY(c.run->omega(pr->dtype, OmegaParams{Om2, m, li, pr->seed, pr->stream_id ^ (uint64_t{1} << 63)}));
  s = gemm(c, pr->prec, true, A, pr->lda, n, m, Om2, l, li, Yt, l, P.tn, P.tn.S > 1 ? c.at<void>(P.part) : nullptr,
           nullptr, true);
  if (s == RSVD_OK) s = reduce_parts(c, P.tn, n, Yt);
  // bases and their triangular factors: Q^T Y = R -> X2, Qt^T Yt = Rt -> X3
  if (s == RSVD_OK) s = orth(c, false, no_split(1), Y, m, Y, X[2]);
  if (s == RSVD_OK) s = orth(c, false, no_split(1), Yt, n, Yt, X[3]);
  if (s != RSVD_OK) return s;
  // M1 = Qt^T Omega -> X0, M2 = Q^T Omegat -> X1 (exact FP64 products)
  RSVD_TRY(cross(c, Yt, l, c.at<void>(P.omega), l, n, li, li, X[0], l, false, true));
  RSVD_TRY(cross(c, Y, l, Om2, l, m, li, li, X[1], l, false, true));
  auto mm = [&](bool trans, const double* a, const double* b, double* out, int64_t ldo, bool accum = false) {
    return gemm(c64, RSVD_NATIVE, trans, a, l, l, l, b, l, li, out, ldo, no_split(l), nullptr, nullptr, false,
                accum);
  };
  auto tr = [&](const double* a, double* out) { return copy2d(c, a, RSVD_F64, l, out, RSVD_F64, l, l, l, true); };
  // G1 = M1 M1^T = W1 D1 W1^T (the plan's eigensolver regions) and G2 = M2 M2^T = W2 D2 W2^T (the
  // second region), both eigensolvers in one launch per stage
  EigParams e = eig_params(c, S);
  EigParams e2 = e;
  {
    const Eig2Layout L2 = eig2_layout(P);
    char* b2 = c.at<char>(P.eig2);
    double* t2 = reinterpret_cast<double*>(b2 + L2.T);
    e2.G = reinterpret_cast<const double*>(b2 + L2.G);
    e2.V = reinterpret_cast<double*>(b2 + L2.V);
    e2.Z = reinterpret_cast<double*>(b2 + L2.Z);
    e2.tri = t2;
    e2.lam = t2 + 3 * l;
    e2.tnorm = t2 + 4 * l;
    e2.flag = reinterpret_cast<int32_t*>(t2 + 4 * l + 1);
    e2.Uh = reinterpret_cast<double*>(b2 + L2.Uh);
    e2.sig = reinterpret_cast<double*>(b2 + L2.sig);
    e2.XU = b2 + L2.XU;
    e2.XV = b2 + L2.XV;
    e2.S = b2 + L2.S;
  }
  for (int side = 0; side < 2; ++side) {
    const double* M = X[side];
    s = tr(M, R3);
    if (s == RSVD_OK) s = mm(false, M, R3, const_cast<double*>(side == 0 ? e.G : e2.G), Lg);
    if (s != RSVD_OK) return s;
  }
  for (int stage = 0; stage < 3; ++stage) RSVD_TRY(launch_eig_pair(stage, e, e2, c.st));
  const double* W1 = e.Uh;
  const double* d1 = e.lam;
  const double* W2 = e2.Uh;
  const double* d2 = e2.lam;
  // C = R M1^T + M2 Rt^T -> R1
  s = tr(X[0], R3);
  if (s == RSVD_OK) s = mm(false, X[2], R3, R1, l);
  if (s == RSVD_OK) s = tr(X[3], R3);
  if (s == RSVD_OK) s = mm(false, X[1], R3, R1, l, true);
  // Chat = W2^T C W1 -> Rt; Bhat = Chat ./ (d2_i + d1_j); B = W2 Bhat W1^T -> R1
  if (s == RSVD_OK) s = mm(true, W2, R1, R2, l);
  if (s == RSVD_OK) s = mm(false, R2, W1, Rt, l);
  if (s != RSVD_OK) return s;
  RSVD_TRY(launch_sylv_div(Rt, l, d2, d1, li, c.st));
  s = mm(false, W2, Rt, R2, l);
  if (s == RSVD_OK) s = tr(W1, R3);
  if (s == RSVD_OK) s = mm(false, R2, R3, R1, l);
  // the SVD of B from its FP64 Gram B B^T: Ub (XU), S, Ub S^-1 (XV)
  if (s == RSVD_OK) s = tr(R1, R3);
  if (s == RSVD_OK) s = mm(false, R1, R3, G, Lg);
  if (s != RSVD_OK) return s;
  for (int stage = 0; stage < 3; ++stage) RSVD_TRY(c.run->eig(stage, e));
  // U = Q Ub_k; V = Qt (B^T Ub_k S_k^-1), B^T rounded to the element type first (RinvT region)
  void* Bt = c.at<void>(P.RinvT);
  void* Vb = X[0];
  s = copy2d(c, R1, RSVD_F64, l, Bt, P.dtype, l, l, l, true);
  if (s == RSVD_OK)
    s = gemm(c, RSVD_NATIVE, false, Bt, l, l, l, e.XV, k, (int32_t)k, Vb, k, no_split(l), nullptr, nullptr);
  if (s == RSVD_OK)
    s = gemm(c, RSVD_NATIVE, false, Y, l, m, l, e.XU, k, (int32_t)k, U, k, no_split(l), nullptr, nullptr);
  if (s == RSVD_OK)
    s = gemm(c, RSVD_NATIVE, false, Yt, l, n, l, Vb, k, (int32_t)k, V, k, no_split(l), nullptr, nullptr);
  return s;
}

rsvd_status gemm_tn_splitk(const Ctx& c, const BwdLayout& L, const void* A, int64_t lda, int64_t rows, int64_t K,
                           const void* X, int64_t ldx, int32_t ncols, void* out, int64_t ldo) {
  return gemm_tn_splitk_into(c, c.at<void>(L.part), A, lda, rows, K, X, ldx, ncols, out, ldo);
}

// out (rows x l, ldo) = gY for Y = Qj R (rows x l): gY = (gQ + Q sym(-gQ^T Q)) R^-T.
rsvd_status qr_adjoint(const Ctx& c, const BwdLayout& L, const void* Qj, const double* Rj, const void* gQ,
                       int64_t rows, void* out, int64_t ldo) {
  const Plan& P = c.P;
  const int64_t l = P.l;
  const int dt = P.dtype;
  rsvd_status s = gemm_tn_splitk(c, L, Qj, l, l, rows, gQ, l, (int32_t)l, c.at<void>(L.Mq), l);  // M = Qj^T gQ
  if (s != RSVD_OK) return s;
  RSVD_TRY(c.run->qr_adj_sym(QrSymParams{c.at<void>(L.Mq), dt, (int32_t)l, c.at<double>(L.Sy)}));
  RSVD_TRY(c.run->tri_inv(TriInvParams{Rj, c.at<double>(L.Rinv), (int32_t)l}));
  s = copy2d(c, c.at<double>(L.Rinv), RSVD_F64, l, c.at<double>(L.W64), RSVD_F64, l, l, l, true);  // R^-T
  if (s != RSVD_OK) return s;
  const Plan p64 = [&] {
    Plan q = P;
    q.dtype = RSVD_F64;
    q.esize = 8;
    return q;
  }();
  const Ctx c64{p64, c.ws, c.st, c.status, c.h, c.run};
  s = gemm(c64, RSVD_NATIVE, false, c.at<double>(L.Sy), l, l, l, c.at<double>(L.W64), l, (int32_t)l,
           c.at<double>(L.SW64), l, no_split(l), nullptr, nullptr);  // S R^-T
  if (s == RSVD_OK) s = copy2d(c, c.at<double>(L.W64), RSVD_F64, l, c.at<void>(L.W), dt, l, l, l, false);
  if (s == RSVD_OK) s = copy2d(c, c.at<double>(L.SW64), RSVD_F64, l, c.at<void>(L.SW), dt, l, l, l, false);
  if (s != RSVD_OK) return s;
  s = gemm(c, RSVD_NATIVE, false, gQ, l, rows, l, c.at<void>(L.W), l, (int32_t)l, out, ldo, no_split(l), nullptr,
           nullptr);
  if (s != RSVD_OK) return s;
  return gemm(c, RSVD_NATIVE, false, Qj, l, rows, l, c.at<void>(L.SW), l, (int32_t)l, out, ldo, no_split(l), nullptr,
              nullptr, false, true);
}

// Y = op(A) X with the split-K partials summed into `out` (rows x l).
rsvd_status stream_apply(const Ctx& c, const rsvd_problem* pr, bool trans, const void* A, const void* X, int64_t ldx,
                         void* out) {
  const Plan& P = c.P;
  const Split& sp = trans ? P.tn : P.nn;
  const int64_t rows = trans ? P.n : P.m;
  const int64_t K = trans ? P.m : P.n;
  rsvd_status s = gemm(c, pr->prec, trans, A, pr->lda, rows, K, X, ldx, (int32_t)P.l, out, P.l, sp,
                       sp.S > 1 ? c.at<void>(P.part) : nullptr, nullptr, true);
  if (s != RSVD_OK) return s;
  return reduce_parts(c, sp, rows, out);
}

// Regions of the kept forward state in an adjoint workspace.
char* kept_Q(const Ctx& c, const BwdLayout& L, int j) {  // Q_j, m x l (j = 0..q)
  return c.at<char>(L.Qs) + (size_t)j * (size_t)(c.P.m * c.P.l) * (size_t)c.P.esize;
}
char* kept_Qt(const Ctx& c, const BwdLayout& L, int j) {  // Qt_j, n x l (j = 1..q)
  return c.at<char>(L.Qts) + (size_t)(j - 1) * (size_t)(c.P.n * c.P.l) * (size_t)c.P.esize;
}
double* kept_R(const Ctx& c, const BwdLayout& L, int j) { return c.at<double>(L.Rs) + (size_t)j * (size_t)(c.P.l * c.P.l); }
double* kept_Rt(const Ctx& c, const BwdLayout& L, int j) {
  return c.at<double>(L.Rts) + (size_t)(j - 1) * (size_t)(c.P.l * c.P.l);
}

// The forward of the adjoint: the range finder and power scheme keeping every
// basis Q_j, Qt_j with its combined triangular factor, B* and the small SVD
// (U~ and sigma in the plan's regions, the k leading singular values in the
// element type to S).  With U and V non-null also the lifts of rsvd_svd,
// U = Q U~_k and V = B* U~_k S_k^-1.  Omega stays in the plan's region.
rsvd_status kept_forward(const Ctx& c, const BwdLayout& L, const rsvd_problem* pr, const void* A, void* U, void* S,
                         void* V) {
  const Plan& P = c.P;
  const int64_t m = P.m, n = P.n, l = P.l, k = P.k;
  void* y = c.at<void>(P.Y);
  void* Bt = c.at<void>(L.Bt);
  rsvd_status s = sketch(c, pr, A, y);
  if (s == RSVD_OK) s = orth(c, P.nn.S > 1, P.nn, y, m, kept_Q(c, L, 0), kept_R(c, L, 0));
  for (int j = 1; j <= L.q && s == RSVD_OK; ++j) {
    s = gemm(c, pr->prec, true, A, pr->lda, n, m, kept_Q(c, L, j - 1), l, (int32_t)l, y, l, P.tn,
             P.tn.S > 1 ? c.at<void>(P.part) : nullptr, nullptr, true);
    if (s == RSVD_OK) s = orth(c, P.tn.S > 1, P.tn, y, n, kept_Qt(c, L, j), kept_Rt(c, L, j));
    if (s == RSVD_OK)
      s = gemm(c, pr->prec, false, A, pr->lda, m, n, kept_Qt(c, L, j), l, (int32_t)l, y, l, P.nn,
               P.nn.S > 1 ? c.at<void>(P.part) : nullptr, nullptr, true);
    if (s == RSVD_OK) s = orth(c, P.nn.S > 1, P.nn, y, m, kept_Q(c, L, j), kept_R(c, L, j));
  }
  if (s == RSVD_OK) s = project_steps(c, pr, A, kept_Q(c, L, L.q), Bt);
  JacobiParams jp;
  if (s == RSVD_OK) s = small_svd(c, Bt, S, jp);
  if (s != RSVD_OK || !U) return s;
  s = gemm(c, RSVD_NATIVE, false, kept_Q(c, L, L.q), l, m, l, jp.XU, k, (int32_t)k, U, k, no_split(l), nullptr,
           nullptr);
  if (s != RSVD_OK) return s;
  return gemm(c, RSVD_NATIVE, false, Bt, l, n, l, jp.XV, k, (int32_t)k, V, k, no_split(l), nullptr, nullptr);
}

// The adjoint proper, from the state kept_forward left in the workspace (which
// it only reads: it may run again on the same state).
rsvd_status adjoint_steps(const Ctx& c, const BwdLayout& L, const rsvd_problem* pr, const void* A, const void* gU,
                          const void* gS, const void* gV, void* gA) {
  const Plan& P = c.P;
  const int64_t m = P.m, n = P.n, l = P.l, k = P.k, Kc = L.Kc;
  const int dt = P.dtype;
  const size_t es = (size_t)P.esize;
  auto Qb = [&](int j) { return kept_Q(c, L, j); };
  auto Qtb = [&](int j) { return kept_Qt(c, L, j); };
  auto Rb = [&](int j) { return kept_R(c, L, j); };
  auto Rtb = [&](int j) { return kept_Rt(c, L, j); };
  char* left = c.at<char>(L.Left);
  char* rightT = c.at<char>(L.RightT);
  void* Bt = c.at<void>(L.Bt);
  rsvd_status s;

  // --- SVD of B and B = Q^T A: gBt = Bt M1 + gV M2, gQ = A gBt + gU U~_k^T
  s = gemm_tn_splitk(c, L, Bt, l, l, n, gV, k, (int32_t)k, c.at<void>(L.T1), k);  // T1 = B gV
  if (s == RSVD_OK) s = gemm_tn_splitk(c, L, Qb(L.q), l, l, m, gU, k, (int32_t)k, c.at<void>(L.T2), k);  // T2 = Q^T gU
  if (s != RSVD_OK) return s;
  SvdAdjParams sa{};
  sa.Uh = c.at<double>(P.Uh);
  sa.sig = c.at<double>(P.sig);
  sa.T1 = c.at<void>(L.T1);
  sa.T2 = c.at<void>(L.T2);
  sa.gS = gS;
  sa.l = (int32_t)l;
  sa.k = (int32_t)k;
  sa.dtype = dt;
  sa.Z = c.at<double>(L.Z);
  sa.M2 = c.at<double>(L.M2_64);
  sa.Ukt = c.at<double>(L.Ukt64);
  RSVD_TRY(c.run->svd_adj_coef(sa));
  Plan p64 = P;
  p64.dtype = RSVD_F64;
  p64.esize = 8;
  const Ctx c64{p64, c.ws, c.st, c.status, c.h, c.run};
  s = copy2d(c, c.at<double>(P.Uh), RSVD_F64, l, c.at<double>(L.UhT), RSVD_F64, l, l, l, true);
  if (s == RSVD_OK)  // W1 = Z U~^T, M1 = U~ W1
    s = gemm(c64, RSVD_NATIVE, false, c.at<double>(L.Z), l, l, l, c.at<double>(L.UhT), l, (int32_t)l,
             c.at<double>(L.W1), l, no_split(l), nullptr, nullptr);
  if (s == RSVD_OK)
    s = gemm(c64, RSVD_NATIVE, false, c.at<double>(P.Uh), l, l, l, c.at<double>(L.W1), l, (int32_t)l,
             c.at<double>(L.M1p64), l, no_split(l), nullptr, nullptr);
  if (s == RSVD_OK) s = copy2d(c, c.at<double>(L.M1p64), RSVD_F64, l, c.at<void>(L.M1p), dt, l, l, l, false);
  if (s == RSVD_OK) s = copy2d(c, c.at<double>(L.M2_64), RSVD_F64, l, c.at<void>(L.M2), dt, l, k, l, false);
  if (s == RSVD_OK) s = copy2d(c, c.at<double>(L.Ukt64), RSVD_F64, l, c.at<void>(L.Ukt), dt, l, k, l, false);
  if (s == RSVD_OK)
    s = gemm(c, RSVD_NATIVE, false, Bt, l, n, l, c.at<void>(L.M1p), l, (int32_t)l, c.at<void>(L.gBt), l,
             no_split(l), nullptr, nullptr);
  if (s == RSVD_OK)
    s = gemm(c, RSVD_NATIVE, false, gV, k, n, k, c.at<void>(L.M2), l, (int32_t)l, c.at<void>(L.gBt), l,
             no_split(k), nullptr, nullptr, false, true);
  // gA block 0: Q_q gBt^T
  if (s == RSVD_OK) s = copy2d(c, Qb(L.q), dt, l, left, dt, Kc, m, l, false);
  if (s == RSVD_OK) s = copy2d(c, c.at<void>(L.gBt), dt, l, rightT, dt, n, n, l, true);
  if (s == RSVD_OK) s = stream_apply(c, pr, false, A, c.at<void>(L.gBt), l, c.at<void>(L.gQ));
  if (s == RSVD_OK)
    s = gemm(c, RSVD_NATIVE, false, gU, k, m, k, c.at<void>(L.Ukt), l, (int32_t)l, c.at<void>(L.gQ), l,
             no_split(k), nullptr, nullptr, false, true);
  if (s != RSVD_OK) return s;

  // --- power steps in reverse, then the sketch
  int64_t blk = 1;
  for (int j = L.q; j >= 1; --j) {
    void* gYj = left + (size_t)(blk * l) * es;  // gY_j = qr adjoint at Q_j, stored as block blk of Left
    s = qr_adjoint(c, L, Qb(j), Rb(j), c.at<void>(L.gQ), m, gYj, Kc);
    if (s == RSVD_OK) s = copy2d(c, Qtb(j), dt, l, rightT + (size_t)(blk * l * n) * es, dt, n, n, l, true);
    ++blk;
    if (s == RSVD_OK) s = stream_apply(c, pr, true, A, gYj, Kc, c.at<void>(L.gQt));  // gQt_j = A^T gY_j
    if (s == RSVD_OK) s = qr_adjoint(c, L, Qtb(j), Rtb(j), c.at<void>(L.gQt), n, c.at<void>(L.gYt), l);
    if (s == RSVD_OK)
      s = copy2d(c, c.at<void>(L.gYt), dt, l, rightT + (size_t)(blk * l * n) * es, dt, n, n, l, true);
    if (s == RSVD_OK) s = copy2d(c, Qb(j - 1), dt, l, left + (size_t)(blk * l) * es, dt, Kc, m, l, false);
    ++blk;
    if (s == RSVD_OK) s = stream_apply(c, pr, false, A, c.at<void>(L.gYt), l, c.at<void>(L.gQ));  // gQ_{j-1}
    if (s != RSVD_OK) return s;
  }
  s = qr_adjoint(c, L, Qb(0), Rb(0), c.at<void>(L.gQ), m, left + (size_t)(blk * l) * es, Kc);  // gY_0
  if (s == RSVD_OK)
    s = copy2d(c, c.at<void>(P.omega), dt, l, rightT + (size_t)(blk * l * n) * es, dt, n, n, l, true);
  if (s != RSVD_OK) return s;

  // --- gA = Left RightT.  BF16 products: one streaming launch over every
  // 128-column chunk (RightT packed once); otherwise 128 columns per launch
  // (FP32 data: the streaming kernels, K = (2q + 2) l in whole 32-deep stages).
  if (P.stream && P.prec != RSVD_NATIVE)
    return gemm(c, pr->prec, false, left, Kc, m, Kc, rightT, n, (int32_t)n, gA, n, no_split(Kc), nullptr, nullptr,
                true, false, c.at<void>(L.gApack), true);
  for (int64_t ch = 0; ch < L.gA_chunks; ++ch) {
    const int64_t c0 = std::min<int64_t>(ch * 128, n - 1);
    const int32_t nc = (int32_t)std::max<int64_t>(1, std::min<int64_t>(128, n - ch * 128));
    const int64_t rows = ch * 128 < n ? m : 0;  // chunks past a narrower problem's n launch nothing
    s = gemm(c, pr->prec, false, left, Kc, rows, Kc, rightT + (size_t)c0 * es, n, nc,
             static_cast<char*>(gA) + (size_t)c0 * es, n, no_split(Kc), nullptr, nullptr, P.stream, false,
             P.stream ? c.at<void>(L.gApack) : nullptr);
    if (s != RSVD_OK) return s;
  }
  return RSVD_OK;
}

// The adjoint with the forward recomputed first.
rsvd_status backward_steps(const Ctx& c, const BwdLayout& L, const rsvd_problem* pr, const void* A, const void* gU,
                           const void* gS, const void* gV, void* gA) {
  const rsvd_status s = kept_forward(c, L, pr, A, nullptr, c.at<void>(L.Sk), nullptr);
  if (s != RSVD_OK) return s;
  return adjoint_steps(c, L, pr, A, gU, gS, gV, gA);
}

struct Prologue {
  rsvd_status status;
  Plan plan;
};

Prologue prologue(rsvd_handle h, const rsvd_problem* pr, const void* ws, size_t ws_bytes) {
  Prologue out{};
  if (!h) {
    out.status = RSVD_E_INVAL;
    return out;
  }
  out.status = validate(pr);
  if (out.status != RSVD_OK) return out;
  out.plan = make_plan(pr);
  if (!ws || ws_bytes < out.plan.total || !aligned16(ws)) {
    out.status = RSVD_E_WORKSPACE;
    return out;
  }
  if (hipSetDevice(h->device) != hipSuccess) out.status = RSVD_E_DEVICE;
  return out;
}

// ---------------------------------------------------------------------------
// Batched calls.

// Per-problem regions of a batched workspace: Q (m x l), Bt (n x l), then the
// problem's own plan.
struct BatchLayout {
  std::vector<Plan> plans;
  std::vector<size_t> base, q_off, bt_off;
  size_t total = 0;
};

// A batch of large matrices (4M elements or more on average) streams A with
// the streaming kernels, one 128-row block of two waves per workgroup; for
// many small matrices the general batched GEMM, with more rows per workgroup
// and no packing pass, is faster.
bool batch_streams(int32_t count, const rsvd_problem* probs) {
  double elems = 0.0;
  for (int32_t i = 0; i < count; ++i) elems += (double)probs[i].m * (double)probs[i].n;
  return elems >= 4194304.0 * count;
}

rsvd_status batch_layout(int32_t count, const rsvd_problem* probs, BatchLayout& L) {
  if (count < 1 || !probs) return RSVD_E_INVAL;
  const rsvd_problem& p0 = probs[0];
  for (int32_t i = 0; i < count; ++i) {
    const rsvd_status v = validate(&probs[i]);
    if (v != RSVD_OK) return v;
    if (probs[i].dtype != p0.dtype || probs[i].prec != p0.prec || probs[i].q != p0.q) return RSVD_E_INVAL;
    if (probs[i].sketch != RSVD_GAUSSIAN) return RSVD_E_UNSUPPORTED;
  }
  const bool stream = batch_streams(count, probs);
  size_t off = 0;
  for (int32_t i = 0; i < count; ++i) {
    const Plan P = make_plan(&probs[i], true, stream);
    const size_t es = (size_t)P.esize;
    L.q_off.push_back(off);
    off += align_up((size_t)P.m * P.l * es);
    L.bt_off.push_back(off);
    off += align_up((size_t)P.n * P.l * es);
    L.base.push_back(off);
    off += P.total;
    L.plans.push_back(P);
  }
  L.total = off;
  return RSVD_OK;
}

}  // namespace

namespace {

// A recorded batch: its identity, the device tables and the replayable graph.
// The tables hold every slot's parameter blocks first, then every slot's block
// map.  Only the parameter blocks hold caller pointers, so a batch whose
// problems and workspace are unchanged but whose caller buffers moved is
// re-pointed by uploading new parameter blocks (from pinned staging memory, on
// the caller's stream); the block maps and the graph stay.
enum BatchKind {
  BATCH_FORWARD = 0, BATCH_BACKWARD = 1, BATCH_FORWARD_KEPT = 2, BATCH_ADJOINT_KEPT = 3,
  SINGLE_FULL = 4  // one problem's four hot-path calls captured as launched (no tables)
};

struct SlotShape {
  int kind, dtype, prec, trans;
  size_t pbytes;
  int64_t nblk;
  bool operator==(const SlotShape& o) const {
    return kind == o.kind && dtype == o.dtype && prec == o.prec && trans == o.trans && pbytes == o.pbytes &&
           nblk == o.nblk;
  }
};

struct BatchPlan {
  int kind = BATCH_FORWARD;
  std::vector<rsvd_problem> probs;
  std::vector<const void*> ptrs;  // the caller buffers of every problem, then the workspace
  std::vector<SlotShape> shape;
  size_t pbytes = 0;                // parameter blocks: tables[0, pbytes)
  void* tables = nullptr;           // device
  void* stage = nullptr;            // pinned host: parameter blocks of the last upload
  hipEvent_t staged = nullptr;      // the last upload from `stage` is complete
  hipEvent_t done = nullptr;        // the last replay is complete
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// A plan's last replay (and its last parameter upload) may still be running on
// the caller's stream when the plan is evicted or replaced: wait for both before
// the graph, the device tables and the pinned staging memory they read go away.
void free_plan(BatchPlan* bp) {
  if (!bp) return;
  if (bp->done) (void)hipEventSynchronize(bp->done);
  if (bp->staged) (void)hipEventSynchronize(bp->staged);
  if (bp->exec) (void)hipGraphExecDestroy(bp->exec);
  if (bp->graph) (void)hipGraphDestroy(bp->graph);
  if (bp->tables) (void)hipFree(bp->tables);
  if (bp->stage) (void)hipHostFree(bp->stage);
  if (bp->staged) (void)hipEventDestroy(bp->staged);
  if (bp->done) (void)hipEventDestroy(bp->done);
  delete bp;
}

// Records one problem's kernel sequence on the given runner.
using Recorder = rsvd_status (*)(const void* ctx, int32_t i, Runner& run);

// The recorded launches of a batch and where they go in the tables.
struct Recorded {
  std::vector<Slot> slots;
  std::vector<SlotShape> shape;
  std::vector<size_t> poff, boff;
  size_t pbytes = 0, bytes = 0;
};

rsvd_status record_batch(int32_t count, int32_t lmax, Recorder rec, const void* ctx, Recorded& R) {
  for (int32_t i = 0; i < count; ++i) {
    RecordRunner rr(R.slots);
    rr.jacobi_maxl_ = jacobi_variant(lmax);
    rr.eig_maxl_ = eig_variant(lmax);
    const rsvd_status s = rec(ctx, i, rr);
    if (s != RSVD_OK) return s == RSVD_E_DEVICE ? RSVD_E_INVAL : s;
    if (rr.cursor() != R.slots.size()) return RSVD_E_INVAL;
  }
  size_t bytes = 0;
  for (const Slot& sl : R.slots) {
    int64_t nb = 0;
    for (int64_t b : sl.blocks) nb += b;
    if (nb > INT32_MAX) return RSVD_E_UNSUPPORTED;
    R.shape.push_back(SlotShape{(int)sl.kind, sl.dtype, sl.prec, sl.trans ? 1 : 0, sl.params.size(), nb});
    R.poff.push_back(bytes);
    bytes = align_up(bytes + sl.params.size());
  }
  R.pbytes = bytes;
  for (const SlotShape& sh : R.shape) {
    R.boff.push_back(bytes);
    bytes = align_up(bytes + (size_t)sh.nblk * sizeof(BlockMap));
  }
  R.bytes = bytes;
  return RSVD_OK;
}

void write_params(const Recorded& R, char* dst) {
  for (size_t s = 0; s < R.slots.size(); ++s)
    std::memcpy(dst + R.poff[s], R.slots[s].params.data(), R.slots[s].params.size());
}

// Launch every slot of a recorded batch on `st` from the device tables.
hipError_t launch_slots(const Recorded& R, const char* dev, hipStream_t st) {
  for (size_t s = 0; s < R.slots.size(); ++s) {
    const Slot& sl = R.slots[s];
    const void* ps = dev + R.poff[s];
    const BlockMap* bm = reinterpret_cast<const BlockMap*>(dev + R.boff[s]);
    const int64_t nb = R.shape[s].nblk;
    hipError_t e = hipSuccess;
    switch (sl.kind) {
      case SK_GEMM:
        e = launch_gemm_batched(sl.dtype, sl.prec, sl.trans, (const GemmParams*)ps, bm, nb, st);
        break;
      case SK_GRAM_PARTIAL:
        e = launch_gram_partial_batched(sl.dtype, (const GramParams*)ps, bm, nb, st);
        break;
      case SK_GRAM_REDUCE:
        e = launch_gram_reduce_batched((const GramReduceParams*)ps, bm, nb, st);
        break;
      case SK_CHOL:
        e = launch_chol_batched((const CholParams*)ps, bm, nb, st);
        break;
      case SK_JACOBI:
        e = launch_jacobi_batched(sl.prec, (const JacobiParams*)ps, bm, nb, st);
        break;
      case SK_OMEGA:
        e = launch_omega_batched(sl.dtype, (const OmegaParams*)ps, bm, nb, st);
        break;
      case SK_TRMM:
        e = launch_trmm_batched((const TrmmParams*)ps, bm, nb, st);
        break;
      case SK_COPY:
        e = launch_copy_batched((const CopyParams*)ps, bm, nb, st);
        break;
      case SK_SUM_PARTS:
        e = launch_sum_parts_batched(sl.dtype, (const GramParams*)ps, bm, nb, st);
        break;
      case SK_SVD_ADJ:
        e = launch_svd_adj_coef_batched((const SvdAdjParams*)ps, bm, nb, st);
        break;
      case SK_QR_SYM:
        e = launch_qr_adj_sym_batched((const QrSymParams*)ps, bm, nb, st);
        break;
      case SK_TRI_INV:
        e = launch_tri_inv_upper_batched((const TriInvParams*)ps, bm, nb, st);
        break;
      case SK_COPY2D:
        e = launch_copy2d_batched((const Copy2dParams*)ps, bm, nb, st);
        break;
      case SK_PACK:
        e = launch_pack_x_batched(sl.prec, (const GemmParams*)ps, bm, nb, st);
        break;
      case SK_STREAM:
        e = launch_stream_gemm_batched(sl.prec, sl.trans, sl.dtype != 0, (const GemmParams*)ps, bm, nb, st);
        break;
      case SK_EIG:
        e = launch_eig_batched(sl.dtype, sl.prec, (const EigParams*)ps, bm, nb, st);
        break;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Workgroup order of one batched step: problems with the longest workgroups
// first (the contraction length of a product, l for the Cholesky and Jacobi
// kernels, the row chunk of a Gram), so that the dispatcher fills the gaps the
// long ones leave with short ones instead of starting a long one last.
int64_t block_weight(const Slot& sl, size_t i) {
  const unsigned char* p = sl.params.data() + i * sl.psize;
  switch (sl.kind) {
    case SK_GEMM:
    case SK_STREAM: {
      const GemmParams& g = *reinterpret_cast<const GemmParams*>(p);
      return std::min(g.K, g.kchunk);
    }
    case SK_GRAM_PARTIAL:
      return reinterpret_cast<const GramParams*>(p)->chunk;
    case SK_CHOL:
      return reinterpret_cast<const CholParams*>(p)->l;
    case SK_JACOBI:
      return reinterpret_cast<const JacobiParams*>(p)->l;
    case SK_EIG:
      return reinterpret_cast<const EigParams*>(p)->l;
    default:
      return 0;
  }
}

void block_order(const Slot& sl, std::vector<int32_t>& order) {
  order.resize(sl.blocks.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int32_t)i;
  std::vector<int64_t> w(order.size());
  for (size_t i = 0; i < w.size(); ++i) w[i] = block_weight(sl, i);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return w[(size_t)a] > w[(size_t)b]; });
}

// Workgroups are dispatched to the 8 XCDs (each with its own L2) round-robin
// in grid order.  A batch of at least 8 problems of one shape gives every
// problem one XCD (longest-processing-time balance of m n), and the block map
// interleaves the XCDs' lists, so all workgroups of a problem share one L2: its
// packed X, and the rows of A that several column chunks read, are fetched
// once per problem instead of once per XCD.  Other batches keep the plain
// longest-first order: with uneven problems a balance of m n leaves steps whose
// work follows l (Cholesky, Jacobi) unbalanced across XCDs (measured slower).
constexpr int kXcds = 8;

std::vector<int32_t> xcd_assignment(int32_t count, const rsvd_problem* probs) {
  std::vector<int32_t> xcd((size_t)count, -1);
  if (count < kXcds) return xcd;
  for (int32_t i = 1; i < count; ++i)
    if (probs[i].m != probs[0].m || probs[i].n != probs[0].n || probs[i].k + probs[i].p != probs[0].k + probs[0].p)
      return xcd;
  std::vector<int32_t> idx((size_t)count);
  for (int32_t i = 0; i < count; ++i) idx[(size_t)i] = i;
  auto work = [&](int32_t i) { return (double)probs[i].m * (double)probs[i].n; };
  std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return work(a) > work(b); });
  double load[kXcds] = {};
  for (const int32_t i : idx) {
    int x = 0;
    for (int y = 1; y < kXcds; ++y)
      if (load[y] < load[x]) x = y;
    xcd[(size_t)i] = x;
    load[x] += work(i);
  }
  return xcd;
}

void fill_block_map(const Slot& sl, const std::vector<int32_t>& xcd, std::vector<int32_t>& order, BlockMap* bm) {
  block_order(sl, order);
  int64_t k = 0;
  if (xcd.empty() || xcd[0] < 0) {
    for (const int32_t i : order)
      for (int64_t b = 0; b < sl.blocks[(size_t)i]; ++b) bm[k++] = BlockMap{i, (int32_t)b};
    return;
  }
  std::vector<std::vector<BlockMap>> lists(kXcds);
  for (const int32_t i : order)
    for (int64_t b = 0; b < sl.blocks[(size_t)i]; ++b) lists[(size_t)xcd[(size_t)i]].push_back(BlockMap{i, (int32_t)b});
  size_t longest = 0;
  for (const auto& li : lists) longest = std::max(longest, li.size());
  for (size_t j = 0; j < longest; ++j)
    for (const auto& li : lists)
      if (j < li.size()) bm[k++] = li[j];
}

// Upload the tables of a recorded batch and capture its launches in a graph.
rsvd_status build_plan(rsvd_handle h, int kind, int32_t count, const rsvd_problem* probs,
                       const std::vector<const void*>& ptrs, const Recorded& R, BatchPlan*& out) {
  std::vector<char> host(R.bytes, 0);
  write_params(R, host.data());
  const std::vector<int32_t> xcd = xcd_assignment(count, probs);
  std::vector<int32_t> order;
  for (size_t s = 0; s < R.slots.size(); ++s)
    fill_block_map(R.slots[s], xcd, order, reinterpret_cast<BlockMap*>(host.data() + R.boff[s]));
  BatchPlan* bp = new (std::nothrow) BatchPlan;
  if (!bp) return RSVD_E_DEVICE;
  bp->kind = kind;
  bp->probs.assign(probs, probs + count);
  bp->ptrs = ptrs;
  bp->shape = R.shape;
  bp->pbytes = R.pbytes;
  rsvd_status st = RSVD_OK;
  if (hipMalloc(&bp->tables, std::max<size_t>(R.bytes, 1)) != hipSuccess ||
      hipMemcpy(bp->tables, host.data(), R.bytes, hipMemcpyHostToDevice) != hipSuccess ||
      hipHostMalloc(&bp->stage, std::max<size_t>(R.pbytes, 1), hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&bp->staged, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&bp->done, hipEventDisableTiming) != hipSuccess)
    st = RSVD_E_DEVICE;
  if (st == RSVD_OK && !h->capture && hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking) != hipSuccess) {
    h->capture = nullptr;
    st = RSVD_E_DEVICE;
  }
  if (st == RSVD_OK) {
    if (hipStreamBeginCapture(h->capture, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      st = RSVD_E_DEVICE;
    } else {
      const hipError_t le = launch_slots(R, static_cast<const char*>(bp->tables), h->capture);
      const hipError_t ce = hipStreamEndCapture(h->capture, &bp->graph);
      if (le != hipSuccess || ce != hipSuccess ||
          hipGraphInstantiate(&bp->exec, bp->graph, nullptr, nullptr, 0) != hipSuccess)
        st = RSVD_E_DEVICE;
    }
  }
  if (st != RSVD_OK) {
    free_plan(bp);
    return st;
  }
  out = bp;
  return RSVD_OK;
}

// Point a plan at new caller buffers: the parameter blocks are rewritten into
// the staging memory (once its previous upload is complete) and uploaded on
// `stream` after the plan's previous replay.  False if the new recording does
// not have the plan's launch structure.
bool repoint_plan(BatchPlan* bp, const Recorded& R, const std::vector<const void*>& ptrs, hipStream_t stream) {
  if (R.shape != bp->shape || R.pbytes != bp->pbytes) return false;
  if (hipEventSynchronize(bp->staged) != hipSuccess) return false;
  write_params(R, static_cast<char*>(bp->stage));
  if (hipStreamWaitEvent(stream, bp->done, 0) != hipSuccess ||
      hipMemcpyAsync(bp->tables, bp->stage, bp->pbytes, hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipEventRecord(bp->staged, stream) != hipSuccess)
    return false;
  bp->ptrs = ptrs;
  return true;
}

bool same_problems(const BatchPlan& bp, int kind, int32_t count, const rsvd_problem* probs) {
  return bp.kind == kind && (int32_t)bp.probs.size() == count &&
         std::memcmp(bp.probs.data(), probs, sizeof(rsvd_problem) * (size_t)count) == 0;
}

// Replay the batch (kind, problems; caller buffers and workspace) on `stream`,
// recording it first if the handle holds no plan for these problems, and
// re-pointing the plan if its buffers or workspace moved.
rsvd_status run_batch(rsvd_handle h, int kind, int32_t count, const rsvd_problem* probs,
                      std::vector<const void*> ptrs, void* ws, Recorder rec, const void* ctx, hipStream_t stream) {
  ptrs.push_back(ws);
  int32_t lmax = 1;
  for (int32_t i = 0; i < count; ++i) lmax = std::max<int32_t>(lmax, probs[i].k + probs[i].p);
  BatchPlan* bp = nullptr;
  size_t at = h->plans.size();
  for (size_t i = 0; i < h->plans.size(); ++i) {
    if (!same_problems(*h->plans[i], kind, count, probs)) continue;
    at = i;
    if (h->plans[i]->ptrs == ptrs) break;
  }
  if (at < h->plans.size()) {
    bp = h->plans[at];
    h->plans.erase(h->plans.begin() + (std::ptrdiff_t)at);
    if (bp->ptrs != ptrs) {
      Recorded R;
      const rsvd_status s = record_batch(count, lmax, rec, ctx, R);
      if (s != RSVD_OK) {
        h->plans.push_back(bp);
        return s;
      }
      if (!repoint_plan(bp, R, ptrs, stream)) {
        free_plan(bp);
        bp = nullptr;
        const rsvd_status b = build_plan(h, kind, count, probs, ptrs, R, bp);
        if (b != RSVD_OK) return b;
      }
    }
  } else {
    Recorded R;
    rsvd_status s = record_batch(count, lmax, rec, ctx, R);
    if (s == RSVD_OK) s = build_plan(h, kind, count, probs, ptrs, R, bp);
    if (s != RSVD_OK) return s;
    if (h->plans.size() >= kMaxPlans) {
      free_plan(h->plans.front());
      h->plans.erase(h->plans.begin());
    }
  }
  h->plans.push_back(bp);  // most recently used last
  RSVD_TRY(hipGraphLaunch(bp->exec, stream));
  RSVD_TRY(hipEventRecord(bp->done, stream));
  return RSVD_OK;
}

// Forward batch: Q, Bt in the batch workspace, the problem's plan after them.
struct ForwardBatch {
  const BatchLayout* L;
  const rsvd_problem* probs;
  const void* const* A;
  void* const *U, *const *S, *const *V;
  char* ws;
  int32_t* status;
};

rsvd_status record_forward(const void* ctx, int32_t i, Runner& run) {
  const ForwardBatch& f = *static_cast<const ForwardBatch*>(ctx);
  const size_t u = (size_t)i;
  const Plan& P = f.L->plans[u];
  const Ctx c{P, f.ws + f.L->base[u], nullptr, f.status, nullptr, &run};
  void* Q = f.ws + f.L->q_off[u];
  void* Bt = f.ws + f.L->bt_off[u];
  const rsvd_problem* pr = &f.probs[u];
  rsvd_status s = range_finder_steps(c, pr, f.A[u], Q, pr->q == 0);
  if (s == RSVD_OK) s = power_steps(c, pr, f.A[u], Q);
  if (s == RSVD_OK) s = project_steps(c, pr, f.A[u], Q, Bt);
  if (s == RSVD_OK) s = svd_steps(c, Bt, Q, f.U[u], f.S[u], f.V[u]);
  return s;
}

// Adjoint batch: each problem's adjoint workspace, one after the other.
struct BackwardBatch {
  std::vector<BwdLayout> L;
  std::vector<size_t> base;
  size_t total = 0;
};

rsvd_status backward_batch_layout(int32_t count, const rsvd_problem* probs, BackwardBatch& B) {
  if (count < 1 || !probs) return RSVD_E_INVAL;
  const rsvd_problem& p0 = probs[0];
  for (int32_t i = 0; i < count; ++i) {
    const rsvd_status v = validate(&probs[i]);
    if (v != RSVD_OK) return v;
    if (probs[i].dtype != p0.dtype || probs[i].prec != p0.prec || probs[i].q != p0.q) return RSVD_E_INVAL;
    if (probs[i].sketch != RSVD_GAUSSIAN) return RSVD_E_UNSUPPORTED;
  }
  const bool stream = batch_streams(count, probs);
  size_t off = 0;
  int64_t chunks = 1;
  for (int32_t i = 0; i < count; ++i) {
    B.L.push_back(bwd_layout(&probs[i], true, stream));
    B.base.push_back(off);
    off += align_up(B.L.back().total);
    chunks = std::max(chunks, B.L.back().gA_chunks);
  }
  for (BwdLayout& L : B.L) L.gA_chunks = chunks;
  B.total = off;
  return RSVD_OK;
}

struct BackwardRecord {
  const BackwardBatch* B;
  const rsvd_problem* probs;
  const void* const *A, *const *gU, *const *gS, *const *gV;
  void* const* gA;
  char* ws;
  int32_t* status;
};

rsvd_status record_backward(const void* ctx, int32_t i, Runner& run) {
  const BackwardRecord& b = *static_cast<const BackwardRecord*>(ctx);
  const size_t u = (size_t)i;
  const BwdLayout& L = b.B->L[u];
  const Ctx c{L.P, b.ws + b.B->base[u], nullptr, b.status, nullptr, &run};
  return backward_steps(c, L, &b.probs[u], b.A[u], b.gU[u], b.gS[u], b.gV[u], b.gA[u]);
}

rsvd_status record_adjoint_kept(const void* ctx, int32_t i, Runner& run) {
  const BackwardRecord& b = *static_cast<const BackwardRecord*>(ctx);
  const size_t u = (size_t)i;
  const BwdLayout& L = b.B->L[u];
  const Ctx c{L.P, b.ws + b.B->base[u], nullptr, b.status, nullptr, &run};
  return adjoint_steps(c, L, &b.probs[u], b.A[u], b.gU[u], b.gS[u], b.gV[u], b.gA[u]);
}

// Kept forward batch: outputs U, S, V, the state in each problem's adjoint workspace.
struct KeptForwardRecord {
  const BackwardBatch* B;
  const rsvd_problem* probs;
  const void* const* A;
  void* const *U, *const *S, *const *V;
  char* ws;
  int32_t* status;
};

rsvd_status record_forward_kept(const void* ctx, int32_t i, Runner& run) {
  const KeptForwardRecord& f = *static_cast<const KeptForwardRecord*>(ctx);
  const size_t u = (size_t)i;
  const BwdLayout& L = f.B->L[u];
  const Ctx c{L.P, f.ws + f.B->base[u], nullptr, f.status, nullptr, &run};
  return kept_forward(c, L, &f.probs[u], f.A[u], f.U[u], f.S[u], f.V[u]);
}

rsvd_status backward_batched_call(rsvd_handle h, int32_t count, const rsvd_problem* probs, const void* const* A,
                                  const void* const* gU, const void* const* gS, const void* const* gV,
                                  void* const* gA, void* ws, size_t ws_bytes, hipStream_t stream, bool kept) {
  if (!h || !A || !gU || !gS || !gV || !gA) return RSVD_E_INVAL;
  BackwardBatch B;
  const rsvd_status v = backward_batch_layout(count, probs, B);
  if (v != RSVD_OK) return v;
  if (!ws || ws_bytes < B.total || !aligned16(ws)) return RSVD_E_WORKSPACE;
  std::vector<const void*> ptrs;
  for (int32_t i = 0; i < count; ++i) {
    if (!A[i] || !gU[i] || !gS[i] || !gV[i] || !gA[i]) return RSVD_E_INVAL;
    ptrs.insert(ptrs.end(), {A[i], gU[i], gS[i], gV[i], gA[i]});
  }
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_E_DEVICE;
  const BackwardRecord r{&B, probs, A, gU, gS, gV, gA, static_cast<char*>(ws), h->status};
  return run_batch(h, kept ? BATCH_ADJOINT_KEPT : BATCH_BACKWARD, count, probs, ptrs, ws,
                   kept ? record_adjoint_kept : record_backward, &r, stream);
}

// One problem's whole rSVD in one workspace: Q (m x l), Bt (n x l), then the
// single-problem plan (with the split of K the four calls use).
struct FullLayout {
  Plan P;
  size_t q_off = 0, bt_off = 0, base = 0, total = 0;
};

FullLayout full_layout(const rsvd_problem* pr) {
  FullLayout F;
  F.P = make_plan(pr);
  const size_t es = (size_t)F.P.esize;
  F.bt_off = align_up((size_t)(F.P.m * F.P.l) * es);
  F.base = F.bt_off + align_up((size_t)(F.P.n * F.P.l) * es);
  F.total = F.base + F.P.total;
  return F;
}

// Capture the four hot-path calls of one problem, launched exactly as the
// single-problem entry points launch them, in a graph.
rsvd_status capture_full(rsvd_handle h, const rsvd_problem* pr, const FullLayout& F, const void* A, void* U,
                         void* S, void* V, char* ws, const std::vector<const void*>& ptrs, BatchPlan*& out) {
  BatchPlan* bp = new (std::nothrow) BatchPlan;
  if (!bp) return RSVD_E_DEVICE;
  bp->kind = SINGLE_FULL;
  bp->probs.assign(pr, pr + 1);
  bp->ptrs = ptrs;
  if (!h->capture && hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking) != hipSuccess) {
    h->capture = nullptr;
    free_plan(bp);
    return RSVD_E_DEVICE;
  }
  if (hipStreamBeginCapture(h->capture, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    free_plan(bp);
    return RSVD_E_DEVICE;
  }
  DirectRunner dr(nullptr, h->capture);  // no timing events inside a graph
  const Ctx c{F.P, ws + F.base, h->capture, h->status, nullptr, &dr};
  void* Q = ws + F.q_off;
  void* Bt = ws + F.bt_off;
  rsvd_status s = range_finder_steps(c, pr, A, Q, pr->q == 0);
  if (s == RSVD_OK) s = power_steps(c, pr, A, Q);
  if (s == RSVD_OK) s = project_steps(c, pr, A, Q, Bt);
  if (s == RSVD_OK) s = svd_steps(c, Bt, Q, U, S, V);
  const hipError_t ce = hipStreamEndCapture(h->capture, &bp->graph);
  if (s == RSVD_OK && (ce != hipSuccess || hipGraphInstantiate(&bp->exec, bp->graph, nullptr, nullptr, 0) != hipSuccess))
    s = RSVD_E_DEVICE;
  if (s != RSVD_OK) {
    free_plan(bp);
    return s;
  }
  out = bp;
  return RSVD_OK;
}

// Shared checks of the single-problem adjoint entry points.
rsvd_status adjoint_prologue(rsvd_handle h, const rsvd_problem* pr, void* ws, size_t ws_bytes, BwdLayout& L) {
  if (!h) return RSVD_E_INVAL;
  const rsvd_status v = validate(pr);
  if (v != RSVD_OK) return v;
  if (pr->sketch != RSVD_GAUSSIAN) return RSVD_E_UNSUPPORTED;
  L = bwd_layout(pr);
  if (!ws || ws_bytes < L.total || !aligned16(ws)) return RSVD_E_WORKSPACE;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_E_DEVICE;
  return RSVD_OK;
}

// ---------------------------------------------------------------------------
// Fixed-precision range finder: Algorithm 4.2 with the samples taken in blocks
// (the remark after Algorithm 4.2) of doubling size (Section 4.3: double the
// guess for the rank at each step).  Block t is first the test of the current
// basis Q by eq. (4.3) -- its projected columns (I - Q Q*) A w are the
// vectors the estimate takes its maximum over -- and is appended if the test
// fails.  The host reads the test statistic after each block.

struct TolLayout {
  int64_t b0 = 0, lmax = 0, L = 0, bmax = 0;  // first block, capacity, test-matrix columns, largest block
  size_t omega = 0, Y = 0, Qb = 0, C = 0, part = 0, base = 0, total = 0;
};

rsvd_problem block_problem(const rsvd_problem* pr, int64_t b) {
  rsvd_problem s = *pr;
  s.k = (int32_t)b;
  s.p = 0;
  s.q = 0;
  return s;
}

rsvd_status tol_layout(const rsvd_problem* pr, int32_t r, TolLayout& T) {
  const rsvd_status v = validate(pr);
  if (v != RSVD_OK) return v;
  if (pr->q != 0 || pr->sketch != RSVD_GAUSSIAN) return RSVD_E_UNSUPPORTED;
  T.b0 = pr->k;
  T.lmax = (int64_t)pr->k + pr->p;
  const int64_t ratio = T.lmax / T.b0;
  if (r < 1 || r > T.b0 || T.lmax % T.b0 != 0 || (ratio & (ratio - 1)) != 0) return RSVD_E_INVAL;
  T.L = T.lmax + r;
  T.bmax = std::max(T.b0, T.lmax / 2);
  const size_t es = pr->dtype == RSVD_F64 ? 8 : 4;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += align_up(std::max<size_t>(bytes, 1));
    return at;
  };
  T.omega = take((size_t)pr->n * (size_t)T.L * es);
  T.Y = take((size_t)pr->m * (size_t)T.bmax * es);
  T.Qb = take((size_t)pr->m * (size_t)T.bmax * es);
  T.C = take((size_t)T.lmax * (size_t)T.bmax * es);
  T.part = take((size_t)kBwdMaxSplit * (size_t)T.lmax * 128 * es);
  T.base = off;
  const rsvd_problem bp = block_problem(pr, T.bmax);
  T.total = T.base + make_plan(&bp).total;
  return RSVD_OK;
}

// Y (m x b) <- (I - Q Q*) Y, twice (the reprojection of Algorithm 4.2, for a block):
// C = Q* Y by the split-K transposed product, then Y += Q (-C).
rsvd_status tol_project(const Ctx& cb, const TolLayout& T, char* ws, const void* Q, int64_t j, void* Y, int64_t b) {
  if (j == 0) return RSVD_OK;
  const int dt = cb.P.dtype;
  void* C = ws + T.C;
  for (int rep = 0; rep < 2; ++rep) {
    rsvd_status s = gemm_tn_splitk_into(cb, ws + T.part, Q, T.lmax, j, cb.P.m, Y, b, (int32_t)b, C, b);
    if (s == RSVD_OK) s = copy2d(cb, C, dt, b, C, dt, b, j, b, false, true);
    if (s == RSVD_OK)
      s = gemm(cb, RSVD_NATIVE, false, Q, T.lmax, cb.P.m, j, C, b, (int32_t)b, Y, b, no_split(j), nullptr, nullptr,
               false, true);
    if (s != RSVD_OK) return s;
  }
  return RSVD_OK;
}

rsvd_status range_finder_tol(rsvd_handle h, const rsvd_problem* pr, const TolLayout& T, double eps, int32_t r,
                             const void* A, void* Q, int32_t* l_out, double* est_out, char* ws, hipStream_t st) {
  const int dt = pr->dtype;
  const size_t es = dt == RSVD_F64 ? 8 : 4;
  DirectRunner dr(h, st);
  char* omega = ws + T.omega;
  void* Y = ws + T.Y;
  void* Qb = ws + T.Qb;
  const double factor = 10.0 * std::sqrt(2.0 / 3.14159265358979323846);
  // every block draws from one n x (lmax + r) Gaussian test matrix, columns in order
  RSVD_TRY(dr.omega(dt, OmegaParams{omega, pr->n, (int32_t)T.L, pr->seed, pr->stream_id}));
  int64_t j = 0, col = 0;
  std::vector<double> diag;
  for (;;) {
    const int64_t b = j == T.lmax ? r : (j == 0 ? T.b0 : j);
    const rsvd_problem bp = block_problem(pr, b);
    const Plan Pb = make_plan(&bp);
    const Ctx cb{Pb, ws + T.base, st, h->status, h, &dr};
    // the block's samples Y = A w for its b fresh test vectors, projected
    rsvd_status s = gemm(cb, pr->prec, false, A, pr->lda, Pb.m, Pb.n, omega + (size_t)col * es, T.L, (int32_t)b, Y, b,
                         Pb.nn, Pb.nn.S > 1 ? cb.at<void>(Pb.part) : nullptr, nullptr, true);
    if (s == RSVD_OK) s = reduce_parts(cb, Pb.nn, Pb.m, Y);
    if (s == RSVD_OK) s = tol_project(cb, T, ws, Q, j, Y, b);
    if (s == RSVD_OK) s = gram(cb, false, no_split(1), Y, Pb.m, nullptr);
    if (s != RSVD_OK) return s;
    col += b;
    // the test statistic: 10 sqrt(2/pi) max_i ||(I - Q Q*) A w_i|| (eq. 4.3)
    diag.assign((size_t)b, 0.0);
    RSVD_TRY(hipMemcpy2DAsync(diag.data(), sizeof(double), cb.at<double>(Pb.G), (size_t)(Pb.Lg + 1) * sizeof(double),
                              sizeof(double), (size_t)b, hipMemcpyDeviceToHost, st));
    RSVD_TRY(hipStreamSynchronize(st));
    double mx = 0.0;
    for (double d : diag) mx = std::max(mx, d);
    const double est = factor * std::sqrt(std::max(mx, 0.0));
    if (!(est > eps) || j == T.lmax) {
      *l_out = (int32_t)j;
      *est_out = est;
      return RSVD_OK;
    }
    // append the block: its orthonormal factor, projected once more and refactored
    s = orth(cb, false, no_split(1), Y, Pb.m, Qb, nullptr);
    if (s == RSVD_OK) s = tol_project(cb, T, ws, Q, j, Qb, b);
    if (s == RSVD_OK && j > 0) s = orth(cb, false, no_split(1), Qb, Pb.m, Qb, nullptr);
    if (s == RSVD_OK) s = copy2d(cb, Qb, dt, b, static_cast<char*>(Q) + (size_t)j * es, dt, T.lmax, Pb.m, b, false);
    if (s != RSVD_OK) return s;
    j += b;
  }
}

}  // namespace

extern "C" {

rsvd_status rsvd_create(rsvd_handle* handle, int device) {
  if (!handle) return RSVD_E_INVAL;
  *handle = nullptr;
  if (hipSetDevice(device) != hipSuccess) return RSVD_E_DEVICE;
  rsvd_handle h = new (std::nothrow) rsvd_handle_s;
  if (!h) return RSVD_E_DEVICE;
  h->device = device;
  h->status = nullptr;
  if (hipMalloc(&h->status, 16) != hipSuccess || hipMemset(h->status, 0, 16) != hipSuccess ||
      hipGetSymbolAddress(reinterpret_cast<void**>(&h->scratch), HIP_SYMBOL(scratch)) != hipSuccess ||
      !h->scratch) {
    if (h->status) (void)hipFree(h->status);
    delete h;
    return RSVD_E_DEVICE;
  }
  *handle = h;
  return RSVD_OK;
}

rsvd_status rsvd_probe_hbm_read(const void* buf, size_t bytes, float* sink, hipStream_t stream) {
  if (!buf || !sink || bytes < 16 || bytes % 16 != 0 || !aligned16(buf)) return RSVD_E_INVAL;
  RSVD_TRY(launch_hbm_read(buf, bytes, sink, stream));
  return RSVD_OK;
}

rsvd_status rsvd_probe_mfma(int32_t kind, int64_t iters, int64_t blocks, float* sink, hipStream_t stream) {
  if (!sink || kind < 0 || kind > 2 || iters < 1 || blocks < 1 || blocks > (int64_t)1 << 20) return RSVD_E_INVAL;
  RSVD_TRY(launch_mfma_loop(kind, iters, blocks, sink, stream));
  return RSVD_OK;
}

rsvd_status rsvd_profile_enable(rsvd_handle h, int32_t capacity) {
  if (!h || capacity < 0) return RSVD_E_INVAL;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_E_DEVICE;
  for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
  h->events.clear();
  h->kinds.clear();
  h->used = 0;
  h->mask = ~0u;
  if (capacity == 0) return RSVD_OK;
  h->events.resize(2 * (size_t)capacity, nullptr);
  h->kinds.resize((size_t)capacity, 0);
  for (auto& e : h->events)
    if (hipEventCreate(&e) != hipSuccess) return RSVD_E_DEVICE;
  return RSVD_OK;
}

rsvd_status rsvd_profile_select(rsvd_handle h, uint32_t mask) {
  if (!h) return RSVD_E_INVAL;
  h->mask = mask;
  return RSVD_OK;
}

rsvd_status rsvd_profile_read(rsvd_handle h, int32_t* launches, double* total_ms) {
  if (!h || !launches || !total_ms) return RSVD_E_INVAL;
  for (int f = 0; f < RSVD_KERNEL_KINDS; ++f) {
    launches[f] = 0;
    total_ms[f] = 0.0;
  }
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_E_DEVICE;
  for (int i = 0; i < h->used; ++i) {
    if (hipEventSynchronize(h->events[2 * i + 1]) != hipSuccess) return RSVD_E_DEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->events[2 * i], h->events[2 * i + 1]) != hipSuccess) return RSVD_E_DEVICE;
    launches[h->kinds[i]] += 1;
    total_ms[h->kinds[i]] += ms;
  }
  h->used = 0;
  return RSVD_OK;
}

rsvd_status rsvd_destroy(rsvd_handle handle) {
  if (!handle) return RSVD_E_INVAL;
  (void)hipSetDevice(handle->device);
  for (BatchPlan* bp : handle->plans) free_plan(bp);
  if (handle->capture) (void)hipStreamDestroy(handle->capture);
  for (hipEvent_t e : handle->events) (void)hipEventDestroy(e);
  (void)hipFree(handle->status);
  delete handle;
  return RSVD_OK;
}

rsvd_status rsvd_validate(const rsvd_problem* problem) { return validate(problem); }

size_t rsvd_workspace_bytes(const rsvd_problem* problem) {
  if (validate(problem) != RSVD_OK) return 0;
  return make_plan(problem).total;
}

const char* rsvd_status_string(rsvd_status s) {
  switch (s) {
    case RSVD_OK: return "ok";
    case RSVD_E_INVAL: return "invalid argument";
    case RSVD_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case RSVD_E_DEVICE: return "HIP device error";
    case RSVD_E_UNSUPPORTED: return "unsupported problem for this library";
    case RSVD_E_BREAKDOWN: return "Cholesky breakdown (shift applied)";
    case RSVD_E_NONFINITE: return "non-finite values encountered";
    case RSVD_E_NOCONV: return "Jacobi SVD did not converge";
  }
  return "unknown status";
}

rsvd_status rsvd_range_finder(rsvd_handle h, const rsvd_problem* pr, const void* A, void* Q, void* ws,
                              size_t ws_bytes, hipStream_t stream) {
  Prologue pro = prologue(h, pr, ws, ws_bytes);
  if (pro.status != RSVD_OK) return pro.status;
  if (!A || !Q) return RSVD_E_INVAL;
  DirectRunner dr(h, stream);
  const Ctx c{pro.plan, static_cast<char*>(ws), stream, h->status, h, &dr};
  return range_finder_steps(c, pr, A, Q, pr->q == 0);
}

rsvd_status rsvd_sketch(rsvd_handle h, const rsvd_problem* pr, const void* A, void* Y, void* ws, size_t ws_bytes,
                        hipStream_t stream) {
  Prologue pro = prologue(h, pr, ws, ws_bytes);
  if (pro.status != RSVD_OK) return pro.status;
  if (!A || !Y) return RSVD_E_INVAL;
  DirectRunner dr(h, stream);
  const Ctx c{pro.plan, static_cast<char*>(ws), stream, h->status, h, &dr};
  rsvd_status s = sketch(c, pr, A, Y);
  if (s != RSVD_OK || pr->sketch != RSVD_GAUSSIAN || c.P.nn.S == 1) return s;
  return reduce_parts(c, c.P.nn, pr->m, Y);
}

rsvd_status rsvd_power_iter(rsvd_handle h, const rsvd_problem* pr, const void* A, void* Q, void* ws,
                            size_t ws_bytes, hipStream_t stream) {
  Prologue pro = prologue(h, pr, ws, ws_bytes);
  if (pro.status != RSVD_OK) return pro.status;
  if (!A || !Q) return RSVD_E_INVAL;
  DirectRunner dr(h, stream);
  const Ctx c{pro.plan, static_cast<char*>(ws), stream, h->status, h, &dr};
  return power_steps(c, pr, A, Q);
}

rsvd_status rsvd_project(rsvd_handle h, const rsvd_problem* pr, const void* A, const void* Q, void* Bt, void* ws,
                         size_t ws_bytes, hipStream_t stream) {
  Prologue pro = prologue(h, pr, ws, ws_bytes);
  if (pro.status != RSVD_OK) return pro.status;
  if (!A || !Q || !Bt) return RSVD_E_INVAL;
  DirectRunner dr(h, stream);
  const Ctx c{pro.plan, static_cast<char*>(ws), stream, h->status, h, &dr};
  return project_steps(c, pr, A, Q, Bt);
}

rsvd_status rsvd_svd(rsvd_handle h, const rsvd_problem* pr, const void* Bt, const void* Q, void* U, void* S,
                     void* V, void* ws, size_t ws_bytes, hipStream_t stream) {
  Prologue pro = prologue(h, pr, ws, ws_bytes);
  if (pro.status != RSVD_OK) return pro.status;
  if (!Bt || !Q || !U || !S || !V) return RSVD_E_INVAL;
  DirectRunner dr(h, stream);
  const Ctx c{pro.plan, static_cast<char*>(ws), stream, h->status, h, &dr};
  return svd_steps(c, Bt, Q, U, S, V);
}

static rsvd_status herm_call(rsvd_handle h, const rsvd_problem* pr, const void* A, const void* Q, void* U,
                             void* Lam, void* ws, size_t ws_bytes, hipStream_t stream, bool nystrom) {
  if (pr && pr->m != pr->n) return RSVD_E_INVAL;
  Prologue pro = prologue(h, pr, ws, ws_bytes);
  if (pro.status != RSVD_OK) return pro.status;
  if (!A || !Q || !U || !Lam) return RSVD_E_INVAL;
  DirectRunner dr(h, stream);
  const Ctx c{pro.plan, static_cast<char*>(ws), stream, h->status, h, &dr};
  return herm_steps(c, pr, A, Q, U, Lam, nystrom);
}

rsvd_status rsvd_eigh(rsvd_handle h, const rsvd_problem* pr, const void* A, const void* Q, void* U, void* Lam,
                      void* ws, size_t ws_bytes, hipStream_t stream) {
  return herm_call(h, pr, A, Q, U, Lam, ws, ws_bytes, stream, false);
}

rsvd_status rsvd_nystrom(rsvd_handle h, const rsvd_problem* pr, const void* A, const void* Q, void* U, void* Lam,
                         void* ws, size_t ws_bytes, hipStream_t stream) {
  return herm_call(h, pr, A, Q, U, Lam, ws, ws_bytes, stream, true);
}

rsvd_status rsvd_eigh_onepass(rsvd_handle h, const rsvd_problem* pr, const void* A, void* U, void* Lam, void* ws,
                              size_t ws_bytes, hipStream_t stream) {
  if (pr && pr->m != pr->n) return RSVD_E_INVAL;
  Prologue pro = prologue(h, pr, ws, ws_bytes);
  if (pro.status != RSVD_OK) return pro.status;
  if (!A || !U || !Lam) return RSVD_E_INVAL;
  DirectRunner dr(h, stream);
  const Ctx c{pro.plan, static_cast<char*>(ws), stream, h->status, h, &dr};
  return onepass_steps(c, pr, A, U, Lam);
}

rsvd_status rsvd_svd_onepass(rsvd_handle h, const rsvd_problem* pr, const void* A, void* U, void* S, void* V,
                             void* ws, size_t ws_bytes, hipStream_t stream) {
  Prologue pro = prologue(h, pr, ws, ws_bytes);
  if (pro.status != RSVD_OK) return pro.status;
  if (!A || !U || !S || !V) return RSVD_E_INVAL;
  DirectRunner dr(h, stream);
  const Ctx c{pro.plan, static_cast<char*>(ws), stream, h->status, h, &dr};
  return svd_onepass_steps(c, pr, A, U, S, V);
}

size_t rsvd_full_workspace_bytes(const rsvd_problem* problem) {
  if (validate(problem) != RSVD_OK) return 0;
  return full_layout(problem).total;
}

rsvd_status rsvd_full(rsvd_handle h, const rsvd_problem* pr, const void* A, void* U, void* S, void* V, void* ws,
                      size_t ws_bytes, hipStream_t stream) {
  if (!h || !A || !U || !S || !V) return RSVD_E_INVAL;
  const rsvd_status v = validate(pr);
  if (v != RSVD_OK) return v;
  const FullLayout F = full_layout(pr);
  if (!ws || ws_bytes < F.total || !aligned16(ws)) return RSVD_E_WORKSPACE;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_E_DEVICE;
  const std::vector<const void*> ptrs{A, U, S, V, ws};
  BatchPlan* bp = nullptr;
  for (size_t i = 0; i < h->plans.size(); ++i) {
    if (same_problems(*h->plans[i], SINGLE_FULL, 1, pr) && h->plans[i]->ptrs == ptrs) {
      bp = h->plans[i];
      h->plans.erase(h->plans.begin() + (std::ptrdiff_t)i);
      break;
    }
  }
  if (!bp) {
    const rsvd_status s = capture_full(h, pr, F, A, U, S, V, static_cast<char*>(ws), ptrs, bp);
    if (s != RSVD_OK) return s;
    if (h->plans.size() >= kMaxPlans) {
      free_plan(h->plans.front());
      h->plans.erase(h->plans.begin());
    }
  }
  h->plans.push_back(bp);  // most recently used last
  RSVD_TRY(hipGraphLaunch(bp->exec, stream));
  return RSVD_OK;
}

rsvd_status rsvd_full_static(rsvd_handle h, const rsvd_problem* pr, const void* A, void* U, void* S, void* V,
                             hipStream_t stream) {
  const rsvd_status v = validate(pr);
  if (v != RSVD_OK) return v;
  const FullLayout F = full_layout(pr);
  if (F.total > (size_t)RSVD_STATIC_SCRATCH_BYTES) return RSVD_E_WORKSPACE;
  if (!h || !h->scratch || !A || !U || !S || !V) return RSVD_E_INVAL;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_E_DEVICE;
  // The kernel sequence of rsvd_full, launched directly (a graph would allocate);
  // nothing in the workspace has to start at zero.
  char* ws = h->scratch;
  DirectRunner dr(h, stream);
  const Ctx c{F.P, ws + F.base, stream, h->status, h, &dr};
  void* Q = ws + F.q_off;
  void* Bt = ws + F.bt_off;
  rsvd_status s = range_finder_steps(c, pr, A, Q, pr->q == 0);
  if (s == RSVD_OK) s = power_steps(c, pr, A, Q);
  if (s == RSVD_OK) s = project_steps(c, pr, A, Q, Bt);
  if (s == RSVD_OK) s = svd_steps(c, Bt, Q, U, S, V);
  return s;
}

size_t rsvd_range_finder_tol_workspace_bytes(const rsvd_problem* problem, int32_t r) {
  TolLayout T;
  return tol_layout(problem, r, T) == RSVD_OK ? T.total : 0;
}

rsvd_status rsvd_range_finder_tol(rsvd_handle h, const rsvd_problem* pr, double eps, int32_t r, const void* A,
                                  void* Q, int32_t* l_out, double* est_out, void* ws, size_t ws_bytes,
                                  hipStream_t stream) {
  TolLayout T;
  const rsvd_status v = tol_layout(pr, r, T);
  if (v != RSVD_OK) return v;
  if (!h || !A || !Q || !l_out || !est_out || !(eps > 0.0) || !std::isfinite(eps)) return RSVD_E_INVAL;
  if (!ws || ws_bytes < T.total || !aligned16(ws)) return RSVD_E_WORKSPACE;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_E_DEVICE;
  return range_finder_tol(h, pr, T, eps, r, A, Q, l_out, est_out, static_cast<char*>(ws), stream);
}

size_t rsvd_backward_workspace_bytes(const rsvd_problem* problem) {
  if (validate(problem) != RSVD_OK || problem->sketch != RSVD_GAUSSIAN) return 0;
  return bwd_layout(problem).total;
}

rsvd_status rsvd_backward(rsvd_handle h, const rsvd_problem* pr, const void* A, const void* gU, const void* gS,
                          const void* gV, void* gA, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!A || !gU || !gS || !gV || !gA) return RSVD_E_INVAL;
  BwdLayout L;
  const rsvd_status v = adjoint_prologue(h, pr, ws, ws_bytes, L);
  if (v != RSVD_OK) return v;
  DirectRunner dr(h, stream);
  const Ctx c{L.P, static_cast<char*>(ws), stream, h->status, h, &dr};
  return backward_steps(c, L, pr, A, gU, gS, gV, gA);
}

rsvd_status rsvd_forward_kept(rsvd_handle h, const rsvd_problem* pr, const void* A, void* U, void* S, void* V,
                              void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!A || !U || !S || !V) return RSVD_E_INVAL;
  BwdLayout L;
  const rsvd_status v = adjoint_prologue(h, pr, ws, ws_bytes, L);
  if (v != RSVD_OK) return v;
  DirectRunner dr(h, stream);
  const Ctx c{L.P, static_cast<char*>(ws), stream, h->status, h, &dr};
  return kept_forward(c, L, pr, A, U, S, V);
}

rsvd_status rsvd_backward_kept(rsvd_handle h, const rsvd_problem* pr, const void* A, const void* gU,
                               const void* gS, const void* gV, void* gA, void* ws, size_t ws_bytes,
                               hipStream_t stream) {
  if (!A || !gU || !gS || !gV || !gA) return RSVD_E_INVAL;
  BwdLayout L;
  const rsvd_status v = adjoint_prologue(h, pr, ws, ws_bytes, L);
  if (v != RSVD_OK) return v;
  DirectRunner dr(h, stream);
  const Ctx c{L.P, static_cast<char*>(ws), stream, h->status, h, &dr};
  return adjoint_steps(c, L, pr, A, gU, gS, gV, gA);
}

size_t rsvd_batched_workspace_bytes(int32_t count, const rsvd_problem* probs) {
  BatchLayout L;
  if (batch_layout(count, probs, L) != RSVD_OK) return 0;
  return L.total;
}

rsvd_status rsvd_batched(rsvd_handle h, int32_t count, const rsvd_problem* probs, const void* const* A,
                         void* const* U, void* const* S, void* const* V, void* ws, size_t ws_bytes,
                         hipStream_t stream) {
  if (!h || !A || !U || !S || !V) return RSVD_E_INVAL;
  BatchLayout L;
  const rsvd_status v = batch_layout(count, probs, L);
  if (v != RSVD_OK) return v;
  if (!ws || ws_bytes < L.total || !aligned16(ws)) return RSVD_E_WORKSPACE;
  std::vector<const void*> ptrs;
  for (int32_t i = 0; i < count; ++i) {
    if (!A[i] || !U[i] || !S[i] || !V[i]) return RSVD_E_INVAL;
    ptrs.insert(ptrs.end(), {A[i], U[i], S[i], V[i]});
  }
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_E_DEVICE;
  const ForwardBatch f{&L, probs, A, U, S, V, static_cast<char*>(ws), h->status};
  return run_batch(h, BATCH_FORWARD, count, probs, ptrs, ws, record_forward, &f, stream);
}

size_t rsvd_backward_batched_workspace_bytes(int32_t count, const rsvd_problem* probs) {
  BackwardBatch B;
  if (backward_batch_layout(count, probs, B) != RSVD_OK) return 0;
  return B.total;
}

rsvd_status rsvd_backward_batched(rsvd_handle h, int32_t count, const rsvd_problem* probs, const void* const* A,
                                  const void* const* gU, const void* const* gS, const void* const* gV,
                                  void* const* gA, void* ws, size_t ws_bytes, hipStream_t stream) {
  return backward_batched_call(h, count, probs, A, gU, gS, gV, gA, ws, ws_bytes, stream, false);
}

rsvd_status rsvd_batched_kept(rsvd_handle h, int32_t count, const rsvd_problem* probs, const void* const* A,
                              void* const* U, void* const* S, void* const* V, void* ws, size_t ws_bytes,
                              hipStream_t stream) {
  if (!h || !A || !U || !S || !V) return RSVD_E_INVAL;
  BackwardBatch B;
  const rsvd_status v = backward_batch_layout(count, probs, B);
  if (v != RSVD_OK) return v;
  if (!ws || ws_bytes < B.total || !aligned16(ws)) return RSVD_E_WORKSPACE;
  std::vector<const void*> ptrs;
  for (int32_t i = 0; i < count; ++i) {
    if (!A[i] || !U[i] || !S[i] || !V[i]) return RSVD_E_INVAL;
    ptrs.insert(ptrs.end(), {A[i], U[i], S[i], V[i]});
  }
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_E_DEVICE;
  const KeptForwardRecord r{&B, probs, A, U, S, V, static_cast<char*>(ws), h->status};
  return run_batch(h, BATCH_FORWARD_KEPT, count, probs, ptrs, ws, record_forward_kept, &r, stream);
}

rsvd_status rsvd_backward_batched_kept(rsvd_handle h, int32_t count, const rsvd_problem* probs,
                                       const void* const* A, const void* const* gU, const void* const* gS,
                                       const void* const* gV, void* const* gA, void* ws, size_t ws_bytes,
                                       hipStream_t stream) {
  return backward_batched_call(h, count, probs, A, gU, gS, gV, gA, ws, ws_bytes, stream, true);
}

rsvd_status rsvd_draw_omega(rsvd_handle h, const rsvd_problem* pr, void* Omega, hipStream_t stream) {
  if (!h || !Omega) return RSVD_E_INVAL;
  const rsvd_status v = validate(pr);
  if (v != RSVD_OK) return v;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_E_DEVICE;
  RSVD_TRY(launch_omega(pr->dtype, Omega, pr->n, pr->k + pr->p, pr->seed, pr->stream_id, stream));
  return RSVD_OK;
}

rsvd_status rsvd_draw_srft(rsvd_handle h, const rsvd_problem* pr, double* d, int32_t* R, hipStream_t stream) {
  if (!h || !d || !R) return RSVD_E_INVAL;
  const rsvd_status v = validate(pr);
  if (v != RSVD_OK) return v;
  if (pr->sketch != RSVD_SRFT) return RSVD_E_INVAL;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_E_DEVICE;
  RSVD_TRY(launch_srft_draw(d, R, pr->n, pr->k + pr->p, pr->seed, pr->stream_id, stream));
  return RSVD_OK;
}

rsvd_status rsvd_orth(rsvd_handle h, const rsvd_problem* pr, int64_t rows, void* Y, double* R, void* ws,
                      size_t ws_bytes, hipStream_t stream) {
  Prologue pro = prologue(h, pr, ws, ws_bytes);
  if (pro.status != RSVD_OK) return pro.status;
  if (!Y || rows < pro.plan.l || rows > pro.plan.Mx) return RSVD_E_INVAL;
  DirectRunner dr(h, stream);
  const Ctx c{pro.plan, static_cast<char*>(ws), stream, h->status, h, &dr};
  return orth(c, false, no_split(1), Y, rows, Y, R);
}

rsvd_status rsvd_device_status(rsvd_handle h, hipStream_t stream, int32_t* flags) {
  if (!h || !flags) return RSVD_E_INVAL;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_E_DEVICE;
  if (hipStreamSynchronize(stream) != hipSuccess) return RSVD_E_DEVICE;
  int32_t v = 0;
  if (hipMemcpy(&v, h->status, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return RSVD_E_DEVICE;
  if (hipMemset(h->status, 0, sizeof(v)) != hipSuccess) return RSVD_E_DEVICE;
  *flags = v;
  return RSVD_OK;
}

}  // extern "C"
