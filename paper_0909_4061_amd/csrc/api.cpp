// Host side of the C ABI declared in include/rsvd.h: argument validation,
// the workspace plan, the split-K choice, and the kernel sequences of the four
// hot-path calls (range finder, power steps, projection, small SVD + lifts).
//
// Every call enqueues its kernels on the caller's stream and returns without
// synchronizing.  Argument errors are found here, before any launch.
#include <algorithm>
#include <new>
#include <vector>

#include "common.hpp"

struct rsvd_handle_s {
  int device;
  int32_t* status;  // device word: RSVD_FLAG_* bits accumulated by the kernels
  // optional launch timing (rsvd_profile_enable)
  std::vector<hipEvent_t> events;  // 2 per record
  std::vector<int> kinds;          // family of each record
  int used = 0;
};

namespace {

using namespace rsvd;

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

struct Split {
  int32_t S;
  int64_t kchunk;
};

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
  Split nn, tn;
  size_t omega, part, Y, Qt, pack, gpart, G, R1, R2, R3, Rt, Rinv, RinvT, XU, XV, Uh, sig, flags, srft_d, srft_R,
      total;
};

bool valid_enum(int32_t v, int32_t lo, int32_t hi) { return v >= lo && v <= hi; }

rsvd_status validate(const rsvd_problem* pr) {
  if (!pr) return RSVD_E_INVAL;
  if (pr->m < 1 || pr->n < 1 || pr->k < 1 || pr->p < 0 || pr->q < 0) return RSVD_E_INVAL;
  if (pr->lda < pr->n) return RSVD_E_INVAL;
  if (!valid_enum(pr->dtype, RSVD_F32, RSVD_F64) || !valid_enum(pr->sketch, RSVD_GAUSSIAN, RSVD_SRFT) ||
      !valid_enum(pr->prec, RSVD_NATIVE, RSVD_BF16X3))
    return RSVD_E_INVAL;
  const int64_t l = (int64_t)pr->k + pr->p;
  if (l > std::min(pr->m, pr->n)) return RSVD_E_INVAL;
  if (l > RSVD_MAX_L) return RSVD_E_UNSUPPORTED;
  if (pr->dtype == RSVD_F64 && pr->prec != RSVD_NATIVE) return RSVD_E_UNSUPPORTED;
  if (pr->sketch == RSVD_SRFT) {
    // One row of A, as n/2 complex values, is transformed in a workgroup's LDS.
    const int64_t nmax = int64_t{2} << (pr->dtype == RSVD_F64 ? SRFT_MAX_LOGN_F64 : SRFT_MAX_LOGN_F32);
    if (pr->q != 0 || pr->n < 8 || pr->n > nmax || (pr->n & (pr->n - 1)) != 0) return RSVD_E_UNSUPPORTED;
  }
  return RSVD_OK;
}

Plan make_plan(const rsvd_problem* pr) {
  Plan P{};
  P.m = pr->m;
  P.n = pr->n;
  P.l = (int64_t)pr->k + pr->p;
  P.k = pr->k;
  P.Mx = std::max(P.m, P.n);
  P.dtype = pr->dtype;
  P.prec = pr->prec;
  P.esize = pr->dtype == RSVD_F64 ? 8 : 4;
  const GemmTile big = gemm_tile(pr->dtype, pr->prec);
  P.Lp = (int32_t)round_up(P.l, big.lp_mult);
  P.Lg = (int32_t)round_up(P.l, 16);
  P.nn = choose_split(P.m, P.n, big);
  P.tn = choose_split(P.n, P.m, big);
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
  P.pack = take(pr->dtype == RSVD_F32 ? (size_t)stream_pack_bytes(P.Mx, P.Lp) : 0);
  P.gpart = take((size_t)ceil_div(P.Mx, GRAM_ROWS) * P.Lg * P.Lg * 8);
  P.G = take((size_t)P.Lg * P.Lg * 8);
  P.R1 = take(ll8);
  P.R2 = take(ll8);
  P.R3 = take(ll8);
  P.Rt = take(ll8);
  P.Rinv = take(ll8);
  P.RinvT = take((size_t)P.l * P.l * es);
  P.XU = take((size_t)P.l * P.k * es);
  P.XV = take((size_t)P.l * P.k * es);
  P.Uh = take(ll8);
  P.sig = take((size_t)P.l * 8);
  P.flags = take(64);
  P.srft_d = take(pr->sketch == RSVD_SRFT ? (size_t)P.n * 8 : 0);
  P.srft_R = take(pr->sketch == RSVD_SRFT ? (size_t)P.l * 4 : 0);
  P.total = off;
  return P;
}

struct Ctx {
  const Plan& P;
  char* ws;
  hipStream_t st;
  int32_t* status;
  rsvd_handle h;
  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(ws + off);
  }
  int32_t* shift_flag() const { return at<int32_t>(P.flags); }
};

#define RSVD_TRY(expr)                          \
  do {                                          \
    if ((expr) != hipSuccess) return RSVD_E_DEVICE; \
  } while (0)

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Brackets one launch with a pair of events when timing is on.
struct Timed {
  rsvd_handle h;
  hipStream_t st;
  int idx = -1;
  Timed(rsvd_handle h_, int kind, hipStream_t st_) : h(h_), st(st_) {
    if (h && h->used < (int)h->kinds.size()) {
      idx = h->used++;
      h->kinds[idx] = kind;
      (void)hipEventRecord(h->events[2 * idx], st);
    }
  }
  ~Timed() {
    if (idx >= 0) (void)hipEventRecord(h->events[2 * idx + 1], st);
  }
};

// op(A) X with the given arithmetic.  With `part` non-null and a split S > 1
// the result is left as partial products; otherwise it is written to `out`.
rsvd_status gemm(const Ctx& c, int prec, bool trans, const void* A, int64_t lda, int64_t rows, int64_t K,
                 const void* X, int64_t ldx, int32_t ncols, void* out, int64_t ldo, const Split& sp, void* part,
                 const int32_t* gate, bool streams_a = false) {
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
  if (g.S > 1 && !part) return RSVD_E_INVAL;
  if (streams_a && c.P.dtype == RSVD_F32) {
    g.Lp = (int32_t)round_up(ncols, 32);
    {
      Timed t_(c.h, RSVD_KERNEL_PACK, c.st);
      RSVD_TRY(launch_pack_x(prec, g, c.at<void>(c.P.pack), c.st));
    }
    Timed t_(c.h, trans ? RSVD_KERNEL_STREAM_TN : RSVD_KERNEL_STREAM_NN, c.st);
    RSVD_TRY(launch_stream_gemm(prec, trans, g, c.at<void>(c.P.pack), c.st));
  } else {
    Timed t_(c.h, streams_a ? (trans ? RSVD_KERNEL_STREAM_TN : RSVD_KERNEL_STREAM_NN) : RSVD_KERNEL_SMALL_GEMM, c.st);
    RSVD_TRY(launch_gemm(c.P.dtype, prec, trans, g, c.st));
  }
  return RSVD_OK;
}

Split no_split(int64_t K) { return Split{1, std::max<int64_t>(K, 1)}; }

// Gram of a rows x l matrix into G (FP64, Lg x Lg upper).  Source: split-K
// partials (summed and stored into `y`) or a stored `y`.
rsvd_status gram(const Ctx& c, bool from_part, const Split& sp, void* y, int64_t rows, const int32_t* gate) {
  GramParams g{};
  g.mode = from_part ? GRAM_FROM_PART : GRAM_FROM_PLAIN;
  g.part = c.at<void>(c.P.part);
  g.S = sp.S;
  g.Lp = c.P.Lp;
  g.yin = y;
  g.yout = y;
  g.ldy = c.P.l;
  g.rows = rows;
  g.l = (int32_t)c.P.l;
  g.Lg = c.P.Lg;
  g.do_gram = 1;
  g.gpart = c.at<double>(c.P.gpart);
  g.gate = gate;
  Timed t_(c.h, RSVD_KERNEL_GRAM, c.st);
  RSVD_TRY(launch_gram_partial(c.P.dtype, g, c.st));
  RSVD_TRY(launch_gram_reduce(g.gpart, ceil_div(rows, GRAM_ROWS), c.P.Lg, c.at<double>(c.P.G), c.status, gate,
                              c.st));
  return RSVD_OK;
}

rsvd_status chol(const Ctx& c, int64_t rows, double* R, bool want_inv, const int32_t* gate, int32_t* shifted) {
  CholParams q{};
  q.G = c.at<double>(c.P.G);
  q.Lg = c.P.Lg;
  q.l = (int32_t)c.P.l;
  q.rows = rows;
  q.R = R;
  q.Rinv = want_inv ? c.at<double>(c.P.Rinv) : nullptr;
  q.RinvT = want_inv ? c.at<void>(c.P.RinvT) : nullptr;
  q.dtype = c.P.dtype;
  q.shifted = shifted;
  q.status = c.status;
  q.gate = gate;
  Timed t_(c.h, RSVD_KERNEL_CHOL, c.st);
  RSVD_TRY(launch_chol(q, c.st));
  return RSVD_OK;
}

// CholeskyQR2 (plus a third pass when a shift was needed) of a rows x l matrix.
// Source: the split-K partials of the GEMM that produced it (from_part; the sum
// is stored into `y`) or `y` itself.  Q (rows x l) may alias y.  If R_out is
// non-null it receives the combined triangular factor.
rsvd_status orth(const Ctx& c, bool from_part, const Split& sp, void* y, int64_t rows, void* Q, double* R_out) {
  const int64_t l = c.P.l;
  int32_t* flag = c.shift_flag();
  RSVD_TRY(launch_fill_i32(flag, 0, 1, c.st));
  double* Rs[3] = {c.at<double>(c.P.R1), c.at<double>(c.P.R2), c.at<double>(c.P.R3)};
  for (int pass = 0; pass < 3; ++pass) {
    const int32_t* gate = pass == 2 ? flag : nullptr;
    const bool src_part = pass == 0 && from_part;
    void* src = pass == 0 ? y : Q;
    rsvd_status s = gram(c, src_part, sp, src, rows, gate);
    if (s != RSVD_OK) return s;
    s = chol(c, rows, Rs[pass], true, gate, pass < 2 ? flag : nullptr);
    if (s != RSVD_OK) return s;
    s = gemm(c, RSVD_NATIVE, false, src, l, rows, l, c.at<void>(c.P.RinvT), l, (int32_t)l, Q, l, no_split(l),
             nullptr, gate);
    if (s != RSVD_OK) return s;
  }
  if (R_out) {
    RSVD_TRY(launch_trmm_upper(Rs[1], Rs[0], R_out, (int32_t)l, nullptr, c.st));
    RSVD_TRY(launch_trmm_upper(Rs[2], R_out, c.at<double>(c.P.Rt), (int32_t)l, flag, c.st));
    RSVD_TRY(launch_copy_f64(c.at<double>(c.P.Rt), R_out, l * l, flag, c.st));
  }
  return RSVD_OK;
}

// Y = A X (NN, rows m) or A^T X (TN, rows n), orthonormalized into Q.
rsvd_status apply_and_orth(const Ctx& c, const rsvd_problem* pr, bool trans, const void* A, const void* X,
                           void* Q) {
  const Plan& P = c.P;
  const Split& sp = trans ? P.tn : P.nn;
  const int64_t rows = trans ? P.n : P.m;
  const int64_t K = trans ? P.m : P.n;
  void* y = c.at<void>(P.Y);
  rsvd_status s = gemm(c, pr->prec, trans, A, pr->lda, rows, K, X, P.l, (int32_t)P.l, y, P.l, sp,
                       sp.S > 1 ? c.at<void>(P.part) : nullptr, nullptr, true);
  if (s != RSVD_OK) return s;
  return orth(c, sp.S > 1, sp, y, rows, Q, nullptr);
}

// Sum the S split-K partial products (rows x l) into `out` in a fixed order.
rsvd_status reduce_parts(const Ctx& c, const Split& sp, int64_t rows, void* out) {
  GramParams g{};
  g.mode = GRAM_FROM_PART;
  g.part = c.at<void>(c.P.part);
  g.S = sp.S;
  g.Lp = c.P.Lp;
  g.yout = out;
  g.ldy = c.P.l;
  g.rows = rows;
  g.l = (int32_t)c.P.l;
  g.Lg = c.P.Lg;
  g.do_gram = 0;
  g.gpart = c.at<double>(c.P.gpart);
  RSVD_TRY(launch_gram_partial(c.P.dtype, g, c.st));
  return RSVD_OK;
}

// Y = A Omega (m x l) for either test matrix, into `y`.
rsvd_status sketch(const Ctx& c, const rsvd_problem* pr, const void* A, void* y) {
  const Plan& P = c.P;
  if (pr->sketch == RSVD_SRFT) {
    double* d = c.at<double>(P.srft_d);
    int32_t* R = c.at<int32_t>(P.srft_R);
    RSVD_TRY(launch_srft_draw(d, R, pr->n, (int32_t)P.l, pr->seed, pr->stream_id, c.st));
    Timed t_(c.h, RSVD_KERNEL_SRFT, c.st);
    RSVD_TRY(launch_srft_rows(pr->dtype, A, pr->lda, pr->m, pr->n, (int32_t)P.l, d, R, y, c.st));
    return RSVD_OK;
  }
  void* omega = c.at<void>(P.omega);
  RSVD_TRY(launch_omega(pr->dtype, omega, pr->n, (int32_t)P.l, pr->seed, pr->stream_id, c.st));
  return gemm(c, pr->prec, false, A, pr->lda, P.m, P.n, omega, P.l, (int32_t)P.l, y, P.l, P.nn,
              P.nn.S > 1 ? c.at<void>(P.part) : nullptr, nullptr, true);
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
  if (hipMalloc(&h->status, 16) != hipSuccess || hipMemset(h->status, 0, 16) != hipSuccess) {
    if (h->status) (void)hipFree(h->status);
    delete h;
    return RSVD_E_DEVICE;
  }
  *handle = h;
  return RSVD_OK;
}

rsvd_status rsvd_profile_enable(rsvd_handle h, int32_t capacity) {
  if (!h || capacity < 0) return RSVD_E_INVAL;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_E_DEVICE;
  for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
  h->events.clear();
  h->kinds.clear();
  h->used = 0;
  if (capacity == 0) return RSVD_OK;
  h->events.resize(2 * (size_t)capacity, nullptr);
  h->kinds.resize((size_t)capacity, 0);
  for (auto& e : h->events)
    if (hipEventCreate(&e) != hipSuccess) return RSVD_E_DEVICE;
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
    case RSVD_E_UNSUPPORTED: return "unsupported problem for this build";
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
  const Ctx c{pro.plan, static_cast<char*>(ws), stream, h->status, h};
  void* y = c.at<void>(c.P.Y);
  const bool parts = pr->sketch == RSVD_GAUSSIAN && c.P.nn.S > 1;
  // Y = A Omega (left as split-K partials for the Gaussian GEMM when S > 1),
  // then CholeskyQR2 (Algorithm 4.1 step 3 / Algorithm 4.5 step 3).
  rsvd_status s = sketch(c, pr, A, y);
  if (s != RSVD_OK) return s;
  return orth(c, parts, c.P.nn, y, pr->m, Q, nullptr);
}

rsvd_status rsvd_sketch(rsvd_handle h, const rsvd_problem* pr, const void* A, void* Y, void* ws, size_t ws_bytes,
                        hipStream_t stream) {
  Prologue pro = prologue(h, pr, ws, ws_bytes);
  if (pro.status != RSVD_OK) return pro.status;
  if (!A || !Y) return RSVD_E_INVAL;
  const Ctx c{pro.plan, static_cast<char*>(ws), stream, h->status, h};
  rsvd_status s = sketch(c, pr, A, Y);
  if (s != RSVD_OK || pr->sketch == RSVD_SRFT || c.P.nn.S == 1) return s;
  return reduce_parts(c, c.P.nn, pr->m, Y);
}

rsvd_status rsvd_power_iter(rsvd_handle h, const rsvd_problem* pr, const void* A, void* Q, void* ws,
                            size_t ws_bytes, hipStream_t stream) {
  Prologue pro = prologue(h, pr, ws, ws_bytes);
  if (pro.status != RSVD_OK) return pro.status;
  if (!A || !Q) return RSVD_E_INVAL;
  const Ctx c{pro.plan, static_cast<char*>(ws), stream, h->status, h};
  void* Qt = c.at<void>(c.P.Qt);
  for (int j = 0; j < pr->q; ++j) {
    rsvd_status s = apply_and_orth(c, pr, true, A, Q, Qt);  // Qt = orth(A^T Q)
    if (s != RSVD_OK) return s;
    s = apply_and_orth(c, pr, false, A, Qt, Q);  // Q = orth(A Qt)
    if (s != RSVD_OK) return s;
  }
  return RSVD_OK;
}

rsvd_status rsvd_project(rsvd_handle h, const rsvd_problem* pr, const void* A, const void* Q, void* Bt, void* ws,
                         size_t ws_bytes, hipStream_t stream) {
  Prologue pro = prologue(h, pr, ws, ws_bytes);
  if (pro.status != RSVD_OK) return pro.status;
  if (!A || !Q || !Bt) return RSVD_E_INVAL;
  const Ctx c{pro.plan, static_cast<char*>(ws), stream, h->status, h};
  const Plan& P = c.P;
  const Split& sp = P.tn;
  rsvd_status s = gemm(c, pr->prec, true, A, pr->lda, P.n, P.m, Q, P.l, (int32_t)P.l, Bt, P.l, sp,
                       sp.S > 1 ? c.at<void>(P.part) : nullptr, nullptr, true);
  if (s != RSVD_OK || sp.S == 1) return s;
  return reduce_parts(c, sp, P.n, Bt);
}

rsvd_status rsvd_svd(rsvd_handle h, const rsvd_problem* pr, const void* Bt, const void* Q, void* U, void* S,
                     void* V, void* ws, size_t ws_bytes, hipStream_t stream) {
  Prologue pro = prologue(h, pr, ws, ws_bytes);
  if (pro.status != RSVD_OK) return pro.status;
  if (!Bt || !Q || !U || !S || !V) return RSVD_E_INVAL;
  const Ctx c{pro.plan, static_cast<char*>(ws), stream, h->status, h};
  const Plan& P = c.P;
  // Gram B B* = Bt^T Bt and its Cholesky factor R (R^T R = B B*).
  rsvd_status s = gram(c, false, no_split(1), const_cast<void*>(Bt), P.n, nullptr);
  if (s != RSVD_OK) return s;
  s = chol(c, P.n, c.at<double>(P.R1), false, nullptr, nullptr);
  if (s != RSVD_OK) return s;
  JacobiParams j{};
  j.R = c.at<double>(P.R1);
  j.l = (int32_t)P.l;
  j.k = (int32_t)P.k;
  j.dtype = P.dtype;
  j.Uh = c.at<double>(P.Uh);
  j.sig = c.at<double>(P.sig);
  j.XU = c.at<void>(P.XU);
  j.XV = c.at<void>(P.XV);
  j.S = S;
  j.status = h->status;
  {
    Timed t_(h, RSVD_KERNEL_JACOBI, stream);
    RSVD_TRY(launch_jacobi(j, stream));
  }
  // U = Q U~_k (m x k), V = Bt U~_k S_k^-1 (n x k)
  s = gemm(c, RSVD_NATIVE, false, Q, P.l, P.m, P.l, j.XU, P.k, (int32_t)P.k, U, P.k, no_split(P.l), nullptr,
           nullptr);
  if (s != RSVD_OK) return s;
  return gemm(c, RSVD_NATIVE, false, Bt, P.l, P.n, P.l, j.XV, P.k, (int32_t)P.k, V, P.k, no_split(P.l), nullptr,
              nullptr);
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
  const Ctx c{pro.plan, static_cast<char*>(ws), stream, h->status, h};
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
