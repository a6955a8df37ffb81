// Host runtime behind the C ABI of include/stau.h: domain validation, FP64
// twiddle / DCT tables (host libm, integer argument reduction), pencil system
// description, device workspaces and the step sequence.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/stau.h"
#include "common.h"
#include "kernels.h"
#include "system.h"

using namespace stau;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(STAU_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));       \
  } while (0)

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// Device scratch of stau_kinetic_energy_noalloc: one array per GPU, held for
// the life of the process.  Host code never uses the array's name as an
// address: each device's address comes from hipGetSymbolAddress, taken once
// per device with that device current (scratch_address).
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
__device__ __align__(256) double2 scratch[kNoAllocBytes / sizeof(double2)];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The scratch address on device `dev`, which must be the current device.
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(STAU_EINVAL, "device ordinal %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(STAU_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return STAU_OK;
}

// exp(-2 pi i t / n) with t reduced modulo n in integers and the angle formed
// in long double.
void fft_table(int64_t n, std::vector<double2>& out) {
  out.resize(n);
  for (int64_t t = 0; t < n; ++t) {
    const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)(t % n) /
                            (long double)n;
    out[t] = make_double2((double)cosl(ang), (double)sinl(ang));
  }
}
// exp(+i pi n / (2 m)), n < m
void dct_table(int64_t m, std::vector<double2>& out) {
  out.resize(m);
  for (int64_t t = 0; t < m; ++t) {
    const long double ang =
        3.14159265358979323846264338327950288L * (long double)t / (2.0L * (long double)m);
    out[t] = make_double2((double)cosl(ang), (double)sinl(ang));
  }
}

// T_n(z_j) on the ascending Gauss grid of m points: z_j = -cos(pi (j + 1/2) / m)
// = cos(pi (2m - 2j - 1) / (2m)), so T_n(z_j) = cos(pi n (2m - 2j - 1) / (2m))
// with the integer argument reduced modulo 4m.
double cheb_T(int64_t n, int64_t j, int64_t m) {
  const int64_t q = (n * (2 * m - 2 * j - 1)) % (4 * m);
  return (double)cosl(3.14159265358979323846264338327950288L * (long double)q / (2.0L * (long double)m));
}

// rows x cols matrix A(i, k) into the 16x16x4 FP64 fragment order
std::vector<double> to_frag(int rows, int cols, const std::vector<double>& A) {
  const int KS = cols / 4;
  std::vector<double> f((size_t)rows * cols);
  for (int rb = 0; rb < rows / 16; ++rb)
    for (int ks = 0; ks < KS; ++ks)
      for (int l = 0; l < 64; ++l)
        f[((size_t)rb * KS + ks) * 64 + l] = A[(size_t)(rb * 16 + l % 16) * cols + ks * 4 + l / 16];
  return f;
}

// BF16 bits of f, rounded to nearest even
uint16_t bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
double bf16_value(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return (double)f;
}

// rows x cols matrix A(i, k) split into three BF16 terms (x = h + m + l) in
// the 16x16x32 BF16 fragment order: lane l of (row block rb, k step ks) holds
// A[16 rb + l mod 16][32 ks + 8 (l / 16) + e], e < 8, at
// ((((rb * KS + ks) * 3 + term) * 64 + l) * 8 + e)
std::vector<uint16_t> to_frag3(int rows, int cols, const std::vector<double>& A) {
  const int KS = cols / 32;
  std::vector<uint16_t> f((size_t)rows * cols * 3);
  for (int rb = 0; rb < rows / 16; ++rb)
    for (int ks = 0; ks < KS; ++ks)
      for (int l = 0; l < 64; ++l)
        for (int e = 0; e < 8; ++e) {
          double x = A[(size_t)(rb * 16 + l % 16) * cols + ks * 32 + 8 * (l / 16) + e];
          for (int term = 0; term < 3; ++term) {
            const uint16_t h = bf16_bits((float)x);
            f[((((size_t)rb * KS + ks) * 3 + term) * 64 + l) * 8 + e] = h;
            x -= bf16_value(h);
          }
        }
  return f;
}

int upload32(const std::vector<double2>& h, float2** d) {
  std::vector<float2> f(h.size());
  for (size_t i = 0; i < h.size(); ++i) f[i] = make_float2((float)h[i].x, (float)h[i].y);
  HIP_TRY(hipMalloc((void**)d, f.size() * sizeof(float2)));
  HIP_TRY(hipMemcpy(*d, f.data(), f.size() * sizeof(float2), hipMemcpyHostToDevice));
  return STAU_OK;
}

template <typename T>
int upload(const std::vector<T>& h, T** d) {
  HIP_TRY(hipMalloc((void**)d, h.size() * sizeof(T)));
  HIP_TRY(hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return STAU_OK;
}

}  // namespace

struct stau_domain {
  stau_domain_desc d{};
  int64_t Ngx = 0, Ngy = 1, Ngz = 0, Px = 0, P = 0, Pa = 0;
  double2 *twz = nullptr, *dctz = nullptr, *twx = nullptr, *twy = nullptr;
  double2 *twz1 = nullptr, *dctz1 = nullptr, *twx1 = nullptr, *twy1 = nullptr;
  float2 *twz32 = nullptr, *dctz32 = nullptr, *twx32 = nullptr, *twy32 = nullptr;
  // z transforms as matrix products (fragment order of the FP64 matrix cores)
  bool mm = false;
  double *Bzfrag = nullptr, *Fzfrag = nullptr, *PLFzfrag = nullptr;
  // mixed path: the same tables split into three BF16 terms
  bool mm16 = false;
  uint16_t *Bz3 = nullptr, *PLFz3 = nullptr;
};

struct stau_pencils {
  stau_domain* dom = nullptr;
  stau_rb_params par{};
  PencilArgs pa{};
  XformArgs xa{};   // dealiased transforms
  XformArgs xa1{};  // scale-1 transforms
  FieldList fl{};      // the explicit term's fields of the step (z transforms)
  YMap ymap{};         // 3-D: the x pass's 12 fields from the backward y pass
  FieldList fl_adj{};  // the adjoint x pass's fields (2-D)
  AccList acc{};
  int64_t n = 0;
  // workspaces
  double2* G = nullptr;    // [NF][M][P]
  double2* G2 = nullptr;   // 3-D: [NF][M][Ngy][Px] after the y pass
  double2* H = nullptr;    // [ne][M][P]
  double2* Bev = nullptr;  // [P][ne][N]
  double2* Gb = nullptr;   // [NF][M][P] adjoint workspace
  // Runge-Kutta stage values (allocated on the first stau_step_rk):
  // F~^{n,j} (j < s - 1), dt L~X^{n,j} (1 <= j < s - 1), M~X^{n,0}; [P][ne][N] each
  double2* rkbuf = nullptr;
  int rk_slots = 0;
  double2* wvec = nullptr; // [N] Chebyshev integration weights of the KE functional
  // Factor storage of one (a0, b0): factor_stride(n) columns per pencil plus
  // factor_slack() zero columns before and after (raw pointers own the memory).
  struct FactorSlot {
    double *Lraw = nullptr, *Uraw = nullptr;
    uint8_t* sraw = nullptr;
    double* Lf = nullptr;
    uint8_t* sl = nullptr;
    double* Uf = nullptr;
    // two-block solve: factors of the leading (T) and trailing (B) blocks,
    // their last-Q elimination steps and the coupling data
    double *LTraw = nullptr, *UTraw = nullptr, *LBraw = nullptr, *UBraw = nullptr;
    uint8_t *sTraw = nullptr, *sBraw = nullptr;
    double *LfT = nullptr, *UfT = nullptr, *LfB = nullptr, *UfB = nullptr;
    uint8_t *slT = nullptr, *slB = nullptr;
    double *tLt = nullptr, *tLb = nullptr, *Rinv = nullptr, *E1 = nullptr, *E2 = nullptr;
    uint8_t *tPt = nullptr, *tPb = nullptr;
    // refined mixed solve: FP32 copies of Lf / Uf (with the same slack), and
    // of both blocks' factors in the two-block layout
    float *L32raw = nullptr, *U32raw = nullptr, *Lf32 = nullptr, *Uf32 = nullptr;
    float *LT32raw = nullptr, *UT32raw = nullptr, *LB32raw = nullptr, *UB32raw = nullptr;
    float *LfT32 = nullptr, *UfT32 = nullptr, *LfB32 = nullptr, *UfB32 = nullptr;
    // sparse records of the factors for the streamed solve (allocated on the
    // first factorisation into the slot where they apply)
    SparseFactors sf{};
    bool sparse = false;
    bool valid = false;
    double a0 = 0.0, b0 = 0.0;
    int64_t stamp = 0;
  } slot[2], slotT[2];    // slotT: factors of the transposed matrices (adjoint)
  FactorSlot evp;         // factors of tau M~ + L~ + L~' (linear stability), whole-band layout
  double* evp_V = nullptr;  // Krylov bases of the stability solver, P (ncv + 1) n doubles
  size_t evp_V_bytes = 0;
  PencilArgs paT{};       // band description of the transposed system
  // two-block solve of the forward system (FP64, 2-D, at most two blocks per
  // compute unit): leading / trailing block descriptions
  bool two = false;
  PencilArgs pt{}, pb{};
  // the same for the transposed system (the adjoint's solves): blocks of A~^T
  bool twoT = false;
  PencilArgs ptT{}, pbT{};
  bool adj_ok = true;  // the transposed band fits the sweep windows
  // mixed domains: the step's solve as FP32 sweeps with one FP64 refinement
  // (single-block layout) instead of the FP64 sweeps
  bool refined = false;
  // adjoint step: a non-blocking side stream (default priority) and the
  // fork / join events of the work it overlaps (created on first use)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int64_t clock = 0;
  // (a0, b0) of the most recent successful stau_factor: stau_solve solves with
  // the factors of this operator (looked up in the cache, refactored if the
  // steps evicted them since)
  bool has_last = false;
  double last_a0 = 0.0, last_b0 = 0.0;
  double* tpl = nullptr;   // device: band templates of the operator (PencilArgs::tpl)
  double* ysp = nullptr;   // device: streamed-solve vectors (PencilArgs::ysp)
  // the step's factors also as sparse records (streamed solve), with their strides
  bool sparse_ok = false;
  SparseFactors sgeom{};
  int* sing = nullptr;     // device: first singular pencil (INT_MAX if none)
  int* flag = nullptr;     // device: non-finite flag
  unsigned int* check = nullptr;  // device: index-check word (builds with STAU_CHECK_BOUNDS)
  double* scratch = nullptr;
  int64_t ws_bytes = 0;
  int64_t last_sing = -1;
  // per-kernel event timing (instrumentation)
  bool timing = false;
  struct Ev {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Ev> events;
};

namespace {
enum Kind { K_ZB = 0, K_XPASS, K_ZF, K_SOLVE, K_FACTOR, K_YPASS, K_NKINDS };

template <typename F>
hipError_t timed(stau_pencils* pen, int kind, hipStream_t st, F&& launch) {
  if (!pen->timing) return launch();
  stau_pencils::Ev ev{kind, nullptr, nullptr};
  hipError_t e = hipEventCreate(&ev.a);
  if (e == hipSuccess) e = hipEventCreate(&ev.b);
  if (e == hipSuccess) e = hipEventRecord(ev.a, st);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(ev.b, st);
  pen->events.push_back(ev);
  return e;
}
}  // namespace

extern "C" {

const char* stau_last_error(void) { return g_err.c_str(); }

int stau_set_kernel_timing(stau_pencils* pen, int enable) {
  if (!pen) return fail(STAU_EINVAL, "null argument");
  pen->timing = enable != 0;
  return STAU_OK;
}

int stau_read_kernel_timing(stau_pencils* pen, double* ms, int64_t* launches, int nkinds) {
  if (!pen || !ms || !launches || nkinds < 0) return fail(STAU_EINVAL, "bad argument");
  HIP_TRY(hipSetDevice(pen->dom->d.device));
  for (int k = 0; k < nkinds; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  int rc = STAU_OK;
  for (auto& ev : pen->events) {
    if (rc == STAU_OK) {
      hipError_t e = hipEventSynchronize(ev.b);
      float t = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&t, ev.a, ev.b);
      if (e != hipSuccess)
        rc = fail(STAU_EHIP, "event timing failed: %s", hipGetErrorString(e));
      else if (ev.kind < nkinds) {
        ms[ev.kind] += t;
        launches[ev.kind] += 1;
      }
    }
    hipEventDestroy(ev.a);
    hipEventDestroy(ev.b);
  }
  pen->events.clear();
  return rc;
}

int stau_create_domain(const stau_domain_desc* desc, stau_domain** out) {
  if (!desc || !out) return fail(STAU_EINVAL, "null argument");
  *out = nullptr;
  const stau_domain_desc& d = *desc;
  if (d.dim != 2 && d.dim != 3) return fail(STAU_EINVAL, "dim=%d must be 2 or 3", d.dim);
  if (d.precision != STAU_FP64 && d.precision != STAU_MIXED)
    return fail(STAU_EINVAL, "precision %d unknown", d.precision);
  if (d.dct_method < STAU_DCT_AUTO || d.dct_method > STAU_DCT_MATMUL)
    return fail(STAU_EINVAL, "dct_method %d unknown", d.dct_method);
  if (d.mixed_solve < STAU_SOLVE_AUTO || d.mixed_solve > STAU_SOLVE_REFINED)
    return fail(STAU_EINVAL, "mixed_solve %d unknown", d.mixed_solve);
  if (d.factor_layout != STAU_FACTORS_AUTO && d.factor_layout != STAU_FACTORS_BAND)
    return fail(STAU_EINVAL, "factor_layout %d unknown", d.factor_layout);
  if (d.dct_method == STAU_DCT_MATMUL && !mm_supported((int)d.Nz))
    return fail(STAU_EUNSUPPORTED, "matrix-product z transforms need Nz a multiple of 32 in [32, 256]");
  if (d.dct_method == STAU_DCT_MATMUL && d.precision == STAU_MIXED && !mm_bf16_supported((int)d.Nz))
    return fail(STAU_EUNSUPPORTED, "mixed-precision matrix-product z transforms need Nz = 64, 128 or 256");
  if (std::fabs(d.dealias - 1.5) > 1e-15) return fail(STAU_EUNSUPPORTED, "dealias must be 1.5");
  if (!is_pow2(d.Nx) || d.Nx < 4 || d.Nx > 4096)
    return fail(STAU_EUNSUPPORTED, "Nx=%lld must be a power of two in [4, 4096]", (long long)d.Nx);
  if (!is_pow2(d.Nz) || d.Nz < 4 || d.Nz > 512)
    return fail(STAU_EUNSUPPORTED, "Nz=%lld must be a power of two in [4, 512]", (long long)d.Nz);
  if (!(d.Lx > 0.0)) return fail(STAU_EINVAL, "Lx must be positive");
  if (d.dim == 3) {
    if (!is_pow2(d.Ny) || d.Ny < 4 || d.Ny > 4096)
      return fail(STAU_EUNSUPPORTED, "Ny=%lld must be a power of two in [4, 4096]", (long long)d.Ny);
    if (!(d.Ly > 0.0)) return fail(STAU_EINVAL, "Ly must be positive");
  }
  HIP_TRY(hipSetDevice(d.device));
  {
    void* sp = nullptr;  // the no-allocation scratch of this device, looked up once
    const int rc0 = scratch_address(d.device, &sp);
    if (rc0) return rc0;
  }
  stau_domain* dom = new (std::nothrow) stau_domain();
  if (!dom) return fail(STAU_ENOMEM, "host allocation failed");
  dom->d = d;
  dom->Ngx = 3 * d.Nx / 2;
  dom->Ngz = 3 * d.Nz / 2;
  dom->Px = d.Nx / 2 + 1;
  dom->P = d.dim == 3 ? dom->Px * d.Ny : dom->Px;
  dom->Pa = d.Nx / 2;
  dom->Ngy = d.dim == 3 ? 3 * d.Ny / 2 : 1;
  std::vector<double2> t;
  int rc;
  fft_table(dom->Ngz, t);
  if ((rc = upload(t, &dom->twz))) goto bad;
  if ((rc = upload32(t, &dom->twz32))) goto bad;
  dct_table(dom->Ngz, t);
  if ((rc = upload(t, &dom->dctz))) goto bad;
  if ((rc = upload32(t, &dom->dctz32))) goto bad;
  fft_table(dom->Ngx, t);
  if ((rc = upload(t, &dom->twx))) goto bad;
  if ((rc = upload32(t, &dom->twx32))) goto bad;
  fft_table(d.Nz, t);
  if ((rc = upload(t, &dom->twz1))) goto bad;
  dct_table(d.Nz, t);
  if ((rc = upload(t, &dom->dctz1))) goto bad;
  fft_table(d.Nx, t);
  if ((rc = upload(t, &dom->twx1))) goto bad;
  dom->mm = mm_supported((int)d.Nz) &&
            (d.dct_method == STAU_DCT_MATMUL || (d.dct_method == STAU_DCT_AUTO && d.Nz <= 64));
  // split-BF16 products for the mixed step: auto takes them for Nz = 64 only
  // (4096x64: 13.8 / 14.4 us against 27.8 / 27.3 for the FP32 FFT); at
  // Nz = 128, 256 the FP32 FFT with half-size tiles is faster (1024x256:
  // 22.5 / 25.3 us against 30.2 / 39.5)
  dom->mm16 = d.precision == STAU_MIXED && mm_bf16_supported((int)d.Nz) &&
              (d.dct_method == STAU_DCT_MATMUL || (d.dct_method == STAU_DCT_AUTO && d.Nz <= 64));
  if (dom->mm || dom->mm16) {
    const int N = (int)d.Nz, M = (int)dom->Ngz;
    std::vector<double> Bz((size_t)M * N), Fz((size_t)N * M), PLFz((size_t)N * M);
    for (int j = 0; j < M; ++j)
      for (int n = 0; n < N; ++n) {
        const double T = cheb_T(n, j, M);
        Bz[(size_t)j * N + n] = T;
        Fz[(size_t)n * M + j] = (n == 0 ? 1.0 : 2.0) / (double)M * T;
      }
    for (int n = 0; n < N; ++n)
      for (int j = 0; j < M; ++j)
        PLFz[(size_t)n * M + j] = (n == 0 ? 1.0 : 0.5) * Fz[(size_t)n * M + j] -
                                  (n + 2 < N ? 0.5 * Fz[(size_t)(n + 2) * M + j] : 0.0);
    if (dom->mm) {
      if ((rc = upload(to_frag(M, N, Bz), &dom->Bzfrag))) goto bad;
      if ((rc = upload(to_frag(N, M, Fz), &dom->Fzfrag))) goto bad;
      if ((rc = upload(to_frag(N, M, PLFz), &dom->PLFzfrag))) goto bad;
    }
    if (dom->mm16) {
      if ((rc = upload(to_frag3(M, N, Bz), &dom->Bz3))) goto bad;
      if ((rc = upload(to_frag3(N, M, PLFz), &dom->PLFz3))) goto bad;
    }
  }
  if (d.dim == 3) {
    fft_table(dom->Ngy, t);
    if ((rc = upload(t, &dom->twy))) goto bad;
    if ((rc = upload32(t, &dom->twy32))) goto bad;
    fft_table(d.Ny, t);
    if ((rc = upload(t, &dom->twy1))) goto bad;
  }
  *out = dom;
  return STAU_OK;
bad:
  stau_destroy_domain(dom);
  return rc;
}

int stau_destroy_domain(stau_domain* dom) {
  if (!dom) return STAU_OK;
  hipSetDevice(dom->d.device);
  hipFree(dom->twz);
  hipFree(dom->dctz);
  hipFree(dom->twx);
  hipFree(dom->twy);
  hipFree(dom->twz1);
  hipFree(dom->dctz1);
  hipFree(dom->twx1);
  hipFree(dom->twz32);
  hipFree(dom->dctz32);
  hipFree(dom->twx32);
  hipFree(dom->twy1);
  hipFree(dom->twy32);
  hipFree(dom->Bzfrag);
  hipFree(dom->Fzfrag);
  hipFree(dom->PLFzfrag);
  hipFree(dom->Bz3);
  hipFree(dom->PLFz3);
  delete dom;
  return STAU_OK;
}

static void free_pencils(stau_pencils* p) {
  if (p->side) (void)hipStreamDestroy(p->side);
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  if (p->ev_join) (void)hipEventDestroy(p->ev_join);
  p->side = nullptr;
  p->ev_fork = p->ev_join = nullptr;
  for (auto& ev : p->events) {
    hipEventDestroy(ev.a);
    hipEventDestroy(ev.b);
  }
  p->events.clear();
  hipFree(p->G);
  hipFree(p->G2);
  hipFree(p->H);
  hipFree(p->Bev);
  hipFree(p->Gb);
  hipFree(p->wvec);
  hipFree(p->rkbuf);
  for (auto* set : {p->slot, p->slotT, &p->evp})
    for (int k = 0; k < (set == &p->evp ? 1 : 2); ++k) {
      auto& f = set[k];
      hipFree(f.Lraw);
      hipFree(f.sraw);
      hipFree(f.Uraw);
      for (void* q : {(void*)f.sf.F, (void*)f.sf.B, (void*)f.sf.lenF, (void*)f.sf.lenB}) (void)hipFree(q);
      for (void* q : {(void*)f.LTraw, (void*)f.UTraw, (void*)f.LBraw, (void*)f.UBraw, (void*)f.sTraw,
                      (void*)f.sBraw, (void*)f.tLt, (void*)f.tLb, (void*)f.Rinv, (void*)f.E1,
                      (void*)f.E2, (void*)f.tPt, (void*)f.tPb, (void*)f.L32raw, (void*)f.U32raw,
                      (void*)f.LT32raw, (void*)f.UT32raw, (void*)f.LB32raw, (void*)f.UB32raw})
        (void)hipFree(q);
      f = stau_pencils::FactorSlot{};
    }
  hipFree(p->tpl);
  hipFree(p->ysp);
  hipFree(p->evp_V);
  hipFree(p->sing);
  hipFree(p->flag);
  hipFree(p->check);
  hipFree(p->scratch);
}

// Allocate (zeroed) factor storage for one slot of the band description pa.
static hipError_t alloc_slot(stau_pencils::FactorSlot& f, const PencilArgs& pa, size_t* bytes,
                             bool fp32 = false) {
  const size_t sk = (size_t)factor_slack();
  const size_t cols = (size_t)pa.P * pa.nst + 2 * sk;
  hipError_t e = hipSuccess;
  auto get = [&](void** ptr, size_t nb) {
    if (e == hipSuccess) e = hipMalloc(ptr, nb);
    if (e == hipSuccess) e = hipMemset(*ptr, 0, nb);
    *bytes += nb;
  };
  get((void**)&f.Lraw, cols * pa.FW * sizeof(double));
  get((void**)&f.Uraw, cols * pa.BW * sizeof(double));
  get((void**)&f.sraw, cols);
  if (fp32) {
    get((void**)&f.L32raw, cols * pa.FW * sizeof(float));
    get((void**)&f.U32raw, cols * pa.BW * sizeof(float));
  }
  if (e != hipSuccess) return e;
  f.Lf = f.Lraw + sk * pa.FW;
  f.Uf = f.Uraw + sk * pa.BW;
  f.sl = f.sraw + sk;
  if (fp32) {
    f.Lf32 = f.L32raw + sk * pa.FW;
    f.Uf32 = f.U32raw + sk * pa.BW;
  }
  return hipSuccess;
}

// Solve window widths for a band: FW >= kl + 1 (8, 16, 32), BW >= kl + ku + 1 (32, 64).
// Allocate (zeroed) two-block factor storage: both blocks' factors (with
// slack), their last-Q steps and the coupling data.
static hipError_t alloc_slot2(stau_pencils::FactorSlot& f, const PencilArgs& pt, const PencilArgs& pb,
                              size_t* bytes, bool fp32 = false) {
  const size_t sk = (size_t)factor_slack();
  const size_t P = (size_t)pt.P, Q = (size_t)pt.Q, K = (size_t)(pt.kl + pt.ku);
  const size_t cT = P * pt.nst + 2 * sk, cB = P * pb.nst + 2 * sk;
  hipError_t e = hipSuccess;
  auto get = [&](void** ptr, size_t nb) {
    if (e == hipSuccess) e = hipMalloc(ptr, nb);
    if (e == hipSuccess) e = hipMemset(*ptr, 0, nb);
    *bytes += nb;
  };
  get((void**)&f.LTraw, cT * pt.FW * sizeof(double));
  get((void**)&f.UTraw, cT * pt.BW * sizeof(double));
  get((void**)&f.sTraw, cT);
  get((void**)&f.LBraw, cB * pb.FW * sizeof(double));
  get((void**)&f.UBraw, cB * pb.BW * sizeof(double));
  get((void**)&f.sBraw, cB);
  get((void**)&f.tLt, P * Q * pt.kl * sizeof(double));
  get((void**)&f.tLb, P * Q * pb.kl * sizeof(double));
  get((void**)&f.tPt, P * Q);
  get((void**)&f.tPb, P * Q);
  get((void**)&f.Rinv, P * K * K * sizeof(double));
  get((void**)&f.E1, P * Q * pt.ku * sizeof(double));
  get((void**)&f.E2, P * Q * pt.kl * sizeof(double));
  if (fp32) {
    get((void**)&f.LT32raw, cT * pt.FW * sizeof(float));
    get((void**)&f.UT32raw, cT * pt.BW * sizeof(float));
    get((void**)&f.LB32raw, cB * pb.FW * sizeof(float));
    get((void**)&f.UB32raw, cB * pb.BW * sizeof(float));
  }
  if (e != hipSuccess) return e;
  if (fp32) {
    f.LfT32 = f.LT32raw + sk * pt.FW;
    f.UfT32 = f.UT32raw + sk * pt.BW;
    f.LfB32 = f.LB32raw + sk * pb.FW;
    f.UfB32 = f.UB32raw + sk * pb.BW;
  }
  f.LfT = f.LTraw + sk * pt.FW;
  f.UfT = f.UTraw + sk * pt.BW;
  f.slT = f.sTraw + sk;
  f.LfB = f.LBraw + sk * pb.FW;
  f.UfB = f.UBraw + sk * pb.BW;
  f.slB = f.sBraw + sk;
  return hipSuccess;
}

static bool window_widths(PencilArgs& pa) {
  pa.FW = pa.kl + 1 <= 8 ? 8 : (pa.kl + 1 <= 16 ? 16 : 32);
  // backward windows of 32, 48 or 64 rows: the stored U columns are BW wide
  pa.BW = pa.kl + pa.ku + 1 <= 32 ? 32 : (pa.kl + pa.ku + 1 <= 48 ? 48 : 64);
  return pa.kl + 1 <= 32 && pa.kl + pa.ku + 1 <= 64;
}

int stau_build_pencils(stau_domain* dom, const stau_rb_params* par, stau_pencils** out) {
  if (!dom || !par || !out) return fail(STAU_EINVAL, "null argument");
  *out = nullptr;
  if (!(par->Ra > 0.0) || !(par->Pr > 0.0)) return fail(STAU_EINVAL, "Ra and Pr must be positive");
  HIP_TRY(hipSetDevice(dom->d.device));
  stau_pencils* pen = new (std::nothrow) stau_pencils();
  if (!pen) return fail(STAU_ENOMEM, "host allocation failed");
  pen->dom = dom;
  pen->par = *par;
  const stau_domain_desc& d = dom->d;
  const int N = (int)d.Nz;
  PencilArgs& pa = pen->pa;
  build_sysdesc(d.dim, N, pa.desc, pa.var_of_abi);
  pa.check = nullptr;
#ifdef STAU_CHECK_BOUNDS
  if (hipMalloc((void**)&pen->check, sizeof(unsigned)) != hipSuccess ||
      hipMemset(pen->check, 0, sizeof(unsigned)) != hipSuccess) {
    hipFree(pen->check);
    delete pen;
    return fail(STAU_ENOMEM, "device allocation failed");
  }
  pa.check = pen->check;
#endif
  pen->n = (int64_t)pa.desc.S * N;
  pa.n = (int)pen->n;
  if (par->n_gamma < 0 || par->n_gamma > kMaxNcc) {
    delete pen;
    return fail(STAU_EINVAL, "n_gamma must be in [0, %d]", kMaxNcc);
  }
  pa.nncc = par->n_gamma;
  for (int k = 0; k < kMaxNcc; ++k) pa.ncc[k] = k < pa.nncc ? par->gamma[k] : 0.0;
  band_widths(pa.desc, pen->n, pa.nncc, &pa.kl, &pa.ku);
  pa.nst = factor_stride(pa.n);
  pa.trans = 0;
  PencilArgs& paT = pen->paT;  // filled below from pa
  if (!window_widths(pa)) {
    delete pen;
    return fail(STAU_EUNSUPPORTED, "band too wide (kl=%d, ku=%d; n_gamma=%d)", pa.kl, pa.ku, pa.nncc);
  }
  pa.P = (int)dom->P;
  pa.Px = (int)dom->Px;
  pa.Ny = (int)d.Ny;
  pa.kappa = std::pow(par->Ra * par->Pr, -0.5);
  pa.nu = std::pow(par->Ra / par->Pr, -0.5);
  pa.buoyancy = par->buoyancy;
  pa.b_bottom = par->b_bottom;
  pa.b_top = par->b_top;
  pa.two_pi_over_Lx = 2.0 * M_PI / d.Lx;
  pa.two_pi_over_Ly = d.dim == 3 ? 2.0 * M_PI / d.Ly : 0.0;
  {
    // band templates of the operator: entries of a0 M~ + b0 L~ separated by
    // their pencil-dependent factors (exact differences of template entries)
    const int n = pa.n, kl = pa.kl, tw = pa.kl + pa.ku + 1;
    const size_t plane = (size_t)n * tw;
    std::vector<double> T(7 * plane, 0.0);
    PencilCoef base{0, 0, pa.kappa, pa.nu, pa.buoyancy, 0, 0, 0, 0, pa.nncc, {}};
    for (int k = 0; k < kMaxNcc; ++k) base.ncc[k] = pa.ncc[k];
    band_templates(pa.desc, base, n, kl, pa.ku, T.data());
    int rc = upload(T, &pen->tpl);
    if (rc) {
      free_pencils(pen);
      delete pen;
      return rc;
    }
    pa.tpl = pen->tpl;
    pa.tkl = kl;
    pa.tw = tw;
    pa.tplane = (long long)plane;
  }
  paT = pa;
  paT.kl = pa.ku;
  paT.ku = pa.kl;
  paT.trans = 1;
  // the transposed operator (adjoint) swaps kl and ku; when it does not fit the
  // sweep windows the adjoint calls are refused for this pencils object
  pen->adj_ok = window_widths(paT);
  pen->refined = d.precision == STAU_MIXED && d.mixed_solve == STAU_SOLVE_REFINED;
  // Two-block solve for 2-D domains with at most two pencils per compute
  // unit: the system splits at m = kb + S k near n / 2 (a leading block that
  // ends inside a mode is singular) into two halves swept in parallel.  In
  // that latency-bound regime the FP64 two-block sweeps beat the mixed
  // solve's two FP32 sweeps and residual, so mixed domains use them too.
  if (d.dim == 2) {
    const int Q = pa.kl + pa.ku, S = pa.desc.S, kb = pa.desc.kb;
    // the trailing block's forward sweep (FW = 32) runs slower per column:
    // its share of the rows is about 48 %
    const int m = kb + S * (int)((0.52 * pa.n - kb) / S), nb = pa.n - m;
    int dev = 0, cus = 0, lds_cu = 0;
    if (m >= Q + 64 && nb >= Q + 64 && hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) ==
            hipSuccess) {
      PencilArgs& t = pen->pt;
      PencilArgs& b = pen->pb;
      t = pa;
      t.blk = 1;
      t.nfull = pa.n;
      t.n = m;
      t.Q = Q;
      t.nst = factor_stride(m);
      b = pa;
      b.blk = 2;
      b.nfull = pa.n;
      b.n = nb;
      b.Q = Q;
      b.kl = pa.ku;
      b.ku = pa.kl;
      b.nst = factor_stride(nb);
      const bool ok = window_widths(t) && window_widths(b) && solve2_supported(t, b);
      // LDS of one two-block solve block (as launch_solve2 sizes it): two
      // blocks must fit a compute unit
      const int FWm = t.FW > b.FW ? t.FW : b.FW, BWm = t.BW > b.BW ? t.BW : b.BW;
      const size_t lds = (size_t)(2 * (t.BW + t.nst + t.FW) + 2 * (b.BW + b.nst + b.FW) + 128 +
                                  (Q * Q + Q * Q + 1) / 2 * 2) * 8 +
                         (size_t)4 * 2 * 16 * (FWm > BWm ? FWm : BWm) * 8;
      pen->two = ok && dom->Pa <= 2 * cus && 2 * lds <= (size_t)lds_cu;
      // transposed blocks: the leading block of A~^T is the transpose of a
      // leading block of A~ (split at a mode boundary), kl and ku swap (the
      // reversed trailing block swaps them back).  Here the leading block has
      // the wide forward window, so it takes the smaller share of the rows.
      const int mT = kb + S * (int)((0.48 * pa.n - kb) / S);
      PencilArgs& tT = pen->ptT;
      PencilArgs& bT = pen->pbT;
      tT = t;
      tT.trans = 1;
      tT.kl = pa.ku;
      tT.ku = pa.kl;
      tT.n = mT;
      tT.nst = factor_stride(mT);
      bT = b;
      bT.trans = 1;
      bT.kl = pa.kl;
      bT.ku = pa.ku;
      bT.n = pa.n - mT;
      bT.nst = factor_stride(pa.n - mT);
      const bool okT = pen->adj_ok && mT >= Q + 64 && pa.n - mT >= Q + 64 && window_widths(tT) &&
                       window_widths(bT) && solve2_supported(tT, bT);
      const int FWmT = tT.FW > bT.FW ? tT.FW : bT.FW, BWmT = tT.BW > bT.BW ? tT.BW : bT.BW;
      const size_t ldsT = (size_t)(2 * (tT.BW + tT.nst + tT.FW) + 2 * (bT.BW + bT.nst + bT.FW) + 128 +
                                   (Q * Q + Q * Q + 1) / 2 * 2) * 8 +
                          (size_t)4 * 2 * 16 * (FWmT > BWmT ? FWmT : BWmT) * 8;
      pen->twoT = okT && dom->Pa <= 2 * cus && 2 * ldsT <= (size_t)lds_cu;
    }
  }

  XformArgs& xa = pen->xa;
  xa.dim = d.dim;
  xa.N = N;
  xa.M = (int)dom->Ngz;
  xa.Nx = (int)d.Nx;
  xa.L = (int)dom->Ngx;
  xa.Pa = (int)dom->Pa;
  xa.Px = (int)dom->Px;
  xa.Ny = (int)d.Ny;
  xa.Ngy = (int)dom->Ngy;
  xa.P = (int)dom->P;
  xa.S = pa.desc.S;
  xa.ne = pa.desc.ne;
  xa.two_pi_over_Lx = pa.two_pi_over_Lx;
  xa.two_pi_over_Ly = pa.two_pi_over_Ly;
  xa.twz = dom->twz;
  xa.dctz = dom->dctz;
  xa.twx = dom->twx;
  xa.twy = dom->twy;
  xa.twz32 = dom->twz32;
  xa.dctz32 = dom->dctz32;
  xa.twx32 = dom->twx32;
  xa.twy32 = dom->twy32;
  pen->xa1 = xa;
  pen->xa1.M = N;
  pen->xa1.L = (int)d.Nx;
  pen->xa1.twz = dom->twz1;
  pen->xa1.dctz = dom->dctz1;
  pen->xa1.twx = dom->twx1;
  pen->xa1.Ngy = d.dim == 3 ? (int)d.Ny : 1;
  pen->xa1.twy = dom->twy1;

  // explicit-term fields through the z (and y) transforms; their x
  // derivatives are formed in the x pass (i kx times the row)
  FieldList& fl = pen->fl;
  if (d.dim == 2) {  // u, w, b, bz, uz, wz
    const int fv[6] = {2, 3, 1, 4, 5, 6};
    fl.nf = 6;
    for (int i = 0; i < 6; ++i) {
      fl.var[i] = fv[i];
      fl.deriv[i] = 0;
    }
  } else {
    // z transforms of u, v, w, b, bz, uz, vz, wz (ABI order p,b,u,v,w,bz,uz,vz,wz);
    // the backward y pass forms the y derivatives (i ky times the column) and
    // hands the x pass u, v, w, b, b_y, bz, u_y, uz, v_y, vz, w_y, wz
    const int fv[8] = {2, 3, 4, 1, 5, 6, 7, 8};
    fl.nf = 8;
    for (int i = 0; i < 8; ++i) {
      fl.var[i] = fv[i];
      fl.deriv[i] = 0;
    }
    const int ys[12] = {0, 1, 2, 3, 3, 4, 0, 5, 1, 6, 2, 7};
    const int yd[12] = {0, 0, 0, 0, 1, 0, 1, 0, 1, 0, 1, 0};
    YMap& ym = pen->ymap;
    ym.n = 12;
    for (int i = 0; i < 12; ++i) {
      ym.src[i] = ys[i];
      ym.der[i] = yd[i];
    }
  }
  // the adjoint x pass recomputes the eight 2-D grid fields with their x
  // derivatives transformed: u, w, b_x, b_z, u_x, u_z, w_x, w_z
  FieldList& fa = pen->fl_adj;
  {
    const int fv[8] = {2, 3, 1, 4, 2, 5, 3, 6};
    const int fd[8] = {0, 0, 1, 0, 1, 0, 1, 0};
    fa.nf = 8;
    for (int i = 0; i < 8; ++i) {
      fa.var[i] = fv[i];
      fa.deriv[i] = fd[i];
    }
  }
  {
    // adjoint of the backward z transform: target variable <- source fields
    AccList& al = pen->acc;
    const int tgt[6] = {2, 3, 1, 4, 5, 6};                 // u, w, b, bz, uz, wz
    const int ns[6] = {2, 2, 1, 1, 1, 1};
    const int sf[6][2] = {{0, 4}, {1, 6}, {2, -1}, {3, -1}, {5, -1}, {7, -1}};
    const int sd[6][2] = {{0, 1}, {0, 1}, {1, 0}, {0, 0}, {0, 0}, {0, 0}};
    al.nt = 6;
    for (int i = 0; i < 6; ++i) {
      al.target[i] = tgt[i];
      al.nsrc[i] = ns[i];
      for (int q = 0; q < 2; ++q) {
        al.src[i][q] = sf[i][q];
        al.deriv[i][q] = sd[i][q];
      }
    }
  }

  const size_t P = dom->P, M = dom->Ngz, ne = pa.desc.ne, n = pen->n;
  // G holds the z-transformed fields (at most 12: also the grid transforms'
  // nine variables and the adjoint's fields), G2 the 12 fields of the 3-D y pass
  const int nfg = d.dim == 3 ? 12 : (fl.nf > pen->fl_adj.nf ? fl.nf : pen->fl_adj.nf);
  const size_t szG = (size_t)nfg * M * P * sizeof(double2);
  const size_t szH = ne * M * P * sizeof(double2);
  const size_t szB = P * ne * N * sizeof(double2);
  const size_t Ngy = (size_t)dom->Ngy, Px = (size_t)dom->Px;
  const size_t szG2 = d.dim == 3 ? (size_t)12 * M * Ngy * Px * sizeof(double2) : 0;
  const size_t szGb = d.dim == 2 ? szG : 0;  // the adjoint is built for 2-D
  const size_t szScratch = (size_t)(3 * N * P + 4 * M * Ngy + 64) * sizeof(double2);
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMalloc((void**)&pen->G, szG);
  if (e == hipSuccess && szG2) e = hipMalloc((void**)&pen->G2, szG2);
  if (e == hipSuccess) e = hipMalloc((void**)&pen->H, szH);
  if (e == hipSuccess) e = hipMalloc((void**)&pen->Bev, szB);
  if (e == hipSuccess && szGb) e = hipMalloc((void**)&pen->Gb, szGb);
  if (e == hipSuccess) e = hipMalloc((void**)&pen->wvec, (size_t)N * sizeof(double2));
  size_t szF = 0;
  for (auto& f : pen->slot)
    if (e == hipSuccess)
      e = pen->two ? alloc_slot2(f, pen->pt, pen->pb, &szF, pen->refined)
                   : alloc_slot(f, pa, &szF, pen->refined);
  if (e == hipSuccess) e = hipMalloc((void**)&pen->sing, sizeof(int));
  if (e == hipSuccess) e = hipMalloc((void**)&pen->flag, sizeof(int));
  if (e == hipSuccess) e = hipMalloc((void**)&pen->scratch, szScratch);
  // the streamed single-block solve keeps each pencil's two real vectors here
  const size_t szY = pen->two ? 0 : (size_t)pa.P * 2 * pa.nst * sizeof(double);
  if (e == hipSuccess && szY) e = hipMalloc((void**)&pen->ysp, szY);
  if (e != hipSuccess) {
    free_pencils(pen);
    delete pen;
    return fail(STAU_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
  }
  pa.ysp = pen->ysp;
  pen->sparse_ok = d.factor_layout == STAU_FACTORS_AUTO && !pen->two && !pen->refined &&
                   sparse_records_apply(pa, &pen->sgeom);
  pen->ws_bytes = (int64_t)(szG + szG2 + szGb + szH + szB + szF + szScratch + szY);
  {
    // KE functional weights: integral over z in [0, 1] of T_m = 1 / (1 - m^2), m even
    std::vector<double2> wv(N);
    for (int m = 0; m < N; ++m)
      wv[m] = make_double2((m & 1) ? 0.0 : 1.0 / (1.0 - (double)m * (double)m), 0.0);
    hipError_t e2 = hipMemcpy(pen->wvec, wv.data(), N * sizeof(double2), hipMemcpyHostToDevice);
    if (e2 != hipSuccess) {
      free_pencils(pen);
      delete pen;
      return fail(STAU_EHIP, "upload failed: %s", hipGetErrorString(e2));
    }
  }
  *out = pen;
  return STAU_OK;
}

int stau_destroy_pencils(stau_pencils* pen) {
  if (!pen) return STAU_OK;
  hipSetDevice(pen->dom->d.device);
  hipDeviceSynchronize();
  free_pencils(pen);
  delete pen;
  return STAU_OK;
}

int stau_query(const stau_pencils* pen, stau_info* info) {
  if (!pen || !info) return fail(STAU_EINVAL, "null argument");
  const stau_domain* dom = pen->dom;
  info->Nx = dom->d.Nx;
  info->Ny = dom->d.dim == 3 ? dom->d.Ny : 1;
  info->Nz = dom->d.Nz;
  info->Ngx = dom->Ngx;
  info->Ngy = dom->Ngy;
  info->Ngz = dom->Ngz;
  info->Px = dom->Px;
  info->P = dom->P;
  info->P_active = dom->d.dim == 2 ? dom->Pa : dom->Pa * (dom->d.Ny - 1);
  info->S = pen->pa.desc.S;
  info->ne = pen->pa.desc.ne;
  info->n = pen->n;
  info->kl = pen->pa.kl;
  info->ku = pen->pa.ku;
  info->state_elems = dom->P * info->S * info->Nz;
  info->hist_elems = 2 * dom->P * 2 * info->ne * info->Nz;
  info->workspace_bytes = pen->ws_bytes;
  return STAU_OK;
}

static int factor_into(stau_pencils* pen, stau_pencils::FactorSlot* set, const PencilArgs& pa,
                       int k, double a0, double b0, hipStream_t st) {
  auto& f = set[k];
  f.valid = false;
  f.sparse = false;
  const int big = 0x7fffffff;
  HIP_TRY(hipMemcpyAsync(pen->sing, &big, sizeof(int), hipMemcpyHostToDevice, st));
  const bool trans = set == pen->slotT;
  const bool two = trans ? pen->twoT : (pen->two && set == pen->slot);
  const PencilArgs& bt = trans ? pen->ptT : pen->pt;
  const PencilArgs& bb = trans ? pen->pbT : pen->pb;
  HIP_TRY(timed(pen, K_FACTOR, st, [&] {
    if (!two) {
      hipError_t e = launch_factor(pa, a0, b0, f.Lf, f.sl, f.Uf, pen->sing, st);
      if (e == hipSuccess && f.L32raw) {  // FP32 copies for the refined mixed solve
        const size_t cols = (size_t)pa.P * pa.nst + 2 * (size_t)factor_slack();
        e = launch_round_f32(f.Lraw, f.L32raw, cols * pa.FW, st);
        if (e == hipSuccess) e = launch_round_f32(f.Uraw, f.U32raw, cols * pa.BW, st);
      }
      if (e == hipSuccess && pen->sparse_ok && set == pen->slot) {
        if (!f.sf.F) {
          // the records are an optimisation: if they cannot be allocated the
          // pencils keep solving on the whole band
          SparseFactors g = pen->sgeom;
          const size_t units = (size_t)pa.P * (pa.nst / kSpU), lens = (size_t)pa.P * kSpLen;
          hipError_t ea = hipMalloc((void**)&g.F, units * g.strideF);
          if (ea == hipSuccess) ea = hipMalloc((void**)&g.B, units * g.strideB);
          if (ea == hipSuccess) ea = hipMalloc((void**)&g.lenF, lens);
          if (ea == hipSuccess) ea = hipMalloc((void**)&g.lenB, lens);
          if (ea == hipSuccess) {
            f.sf = g;
            pen->ws_bytes += (int64_t)(units * (g.strideF + g.strideB) + 2 * lens);
          } else {
            for (void* q : {(void*)g.F, (void*)g.B, (void*)g.lenF, (void*)g.lenB}) (void)hipFree(q);
            (void)hipGetLastError();  // clear the failed allocation's error
            pen->sparse_ok = false;
            for (auto& o : pen->slot) o.sparse = false;
          }
        }
        if (pen->sparse_ok) {
          e = launch_sparse_records(pa, f.Lf, f.sl, f.Uf, f.sf, st);
          f.sparse = e == hipSuccess;
        }
      }
      return e;
    }
    hipError_t e = launch_factor(bt, a0, b0, f.LfT, f.slT, f.UfT, pen->sing, st, f.tLt, f.tPt);
    if (e == hipSuccess) e = launch_factor(bb, a0, b0, f.LfB, f.slB, f.UfB, pen->sing, st, f.tLb, f.tPb);
    if (e == hipSuccess)
      e = launch_coupling(bt, bb, a0, b0, f.tLt, f.tPt, f.tLb, f.tPb, f.UfT, f.UfB, f.Rinv, f.E1, f.E2,
                          pen->sing, st);
    if (e == hipSuccess && f.LT32raw) {  // FP32 copies for the refined mixed solve
      const size_t sk2 = 2 * (size_t)factor_slack();
      const size_t cT = (size_t)bt.P * bt.nst + sk2, cB = (size_t)bb.P * bb.nst + sk2;
      e = launch_round_f32(f.LTraw, f.LT32raw, cT * bt.FW, st);
      if (e == hipSuccess) e = launch_round_f32(f.UTraw, f.UT32raw, cT * bt.BW, st);
      if (e == hipSuccess) e = launch_round_f32(f.LBraw, f.LB32raw, cB * bb.FW, st);
      if (e == hipSuccess) e = launch_round_f32(f.UBraw, f.UB32raw, cB * bb.BW, st);
    }
    return e;
  }));
  int h = big;
  HIP_TRY(hipMemcpyAsync(&h, pen->sing, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (h != big) {
    pen->last_sing = h;
    return fail(STAU_ESINGULAR, "zero or non-finite pivot in pencil %d", h);
  }
  f.valid = true;
  f.a0 = a0;
  f.b0 = b0;
  f.stamp = ++pen->clock;
  pen->last_sing = -1;
  return STAU_OK;
}

// Factors for (a0, b0): a cached slot if one matches, else refactor the least
// recently used slot (two slots: the SBDF1 and SBDF2 operators of a run).
// trans selects the factors of the transposed matrices (allocated on first use).
static int factors_for(stau_pencils* pen, double a0, double b0, hipStream_t st,
                       stau_pencils::FactorSlot** out, bool trans = false) {
  stau_pencils::FactorSlot* set = trans ? pen->slotT : pen->slot;
  const PencilArgs& pa = trans ? pen->paT : pen->pa;
  for (int q = 0; q < 2; ++q)
    if (set[q].valid && set[q].a0 == a0 && set[q].b0 == b0) {
      set[q].stamp = ++pen->clock;
      *out = &set[q];
      return STAU_OK;
    }
  int k = set[0].stamp <= set[1].stamp ? 0 : 1;
  if (!set[0].valid) k = 0;
  else if (!set[1].valid) k = 1;
  if (!set[k].Lraw && !set[k].LTraw) {  // (two-block slots are allocated with the pencils)
    size_t bytes = 0;
    hipError_t e = (trans && pen->twoT) ? alloc_slot2(set[k], pen->ptT, pen->pbT, &bytes)
                                        : alloc_slot(set[k], pa, &bytes, !trans && pen->refined);
    if (e != hipSuccess) return fail(STAU_ENOMEM, "factor allocation failed: %s", hipGetErrorString(e));
    pen->ws_bytes += (int64_t)bytes;
  }
  int rc = factor_into(pen, set, pa, k, a0, b0, st);
  if (rc) return rc;
  *out = &set[k];
  return STAU_OK;
}

int stau_factor(stau_pencils* pen, double a0, double b0, void* stream) {
  if (!pen) return fail(STAU_EINVAL, "null argument");
  if (!std::isfinite(a0) || !std::isfinite(b0)) return fail(STAU_EINVAL, "non-finite a0/b0");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(pen->dom->d.device));
  int k = pen->slot[0].stamp <= pen->slot[1].stamp ? 0 : 1;
  for (int q = 0; q < 2; ++q)
    if (pen->slot[q].valid && pen->slot[q].a0 == a0 && pen->slot[q].b0 == b0) k = q;
  int rc = factor_into(pen, pen->slot, pen->pa, k, a0, b0, st);
  pen->has_last = rc == STAU_OK;
  pen->last_a0 = a0;
  pen->last_b0 = b0;
  return rc;
}

int64_t stau_last_singular_pencil(const stau_pencils* pen) { return pen ? pen->last_sing : -1; }

static void sbdf(int64_t it, double dt, double dtp, double* a0, double* a1, double* a2, double* b0,
                 double* c1, double* c2) {
  if (it == 0) {
    *a0 = 1.0 / dt;
    *a1 = -1.0 / dt;
    *a2 = 0.0;
    *b0 = 1.0;
    *c1 = 1.0;
    *c2 = 0.0;
    return;
  }
  const double w = dt / dtp;
  *a0 = (1.0 + 2.0 * w) / ((1.0 + w) * dt);
  *a1 = -(1.0 + w) / dt;
  *a2 = w * w / ((1.0 + w) * dt);
  *b0 = 1.0;
  *c1 = 1.0 + w;
  *c2 = -w;
}

// Grid-space explicit term up to the z forward transform: H[e][jz][p].
// 2-D: z backward, fused x pass.  3-D: z backward, y backward, fused x pass,
// y forward (the x-pass output H2 reuses G, the y-forward output goes to H).
static hipError_t explicit_term(stau_pencils* pen, const void* X, hipStream_t st, bool mixed) {
  const bool mm = pen->dom->mm && !mixed, mm16 = pen->dom->mm16 && mixed;
  hipError_t e = timed(pen, K_ZB, st, [&] {
    if (mm) return launch_zb_mm(pen->xa, pen->fl, X, pen->G, pen->dom->Bzfrag, st);
    if (mm16) return launch_zb_bf16(pen->xa, pen->fl, X, pen->G, pen->dom->Bz3, st);
    return launch_zb(pen->xa, pen->fl, X, pen->G, st, mixed, true);
  });
  if (e != hipSuccess) return e;
  if (pen->dom->d.dim == 2)
    return timed(pen, K_XPASS, st, [&] { return launch_xpass(pen->xa, pen->G, pen->H, st, mixed); });
  e = timed(pen, K_YPASS, st,
            [&] { return launch_ypass(pen->xa, +1, pen->ymap.n, pen->G, pen->G2, st, mixed, 0.0, &pen->ymap); });
  if (e != hipSuccess) return e;
  e = timed(pen, K_XPASS, st, [&] { return launch_xpass3(pen->xa, pen->G2, pen->G, st, mixed); });
  if (e != hipSuccess) return e;
  return timed(pen, K_YPASS, st,
               [&] { return launch_ypass(pen->xa, -1, pen->pa.desc.ne, pen->G, pen->H, st, mixed); });
}

// Pencil solve of the step with the factors fs of (a0, b0): in mixed domains
// with the refined solve, FP32 sweeps and one FP64 refinement; otherwise FP64,
// the two-block solve where it applies, else the single-block solve.
static hipError_t solve_launch(stau_pencils* pen, const stau_pencils::FactorSlot* fs, double a0,
                               double b0, const double2* B, void* X, hipStream_t st, bool mixed) {
  if (mixed && pen->refined && pen->two && fs->LfT32) {
    PencilArgs pt = pen->pt, pb = pen->pb;
    pt.refine_a0 = pb.refine_a0 = a0;
    pt.refine_b0 = pb.refine_b0 = b0;
    return launch_solve2_refined(pt, pb, B, fs->LfT32, fs->slT, fs->UfT32, fs->LfB32, fs->slB, fs->UfB32,
                                 fs->Rinv, fs->E1, fs->E2, X, st);
  }
  if (mixed && pen->refined && fs->Lf32) {
    PencilArgs pr = pen->pa;
    pr.refine_a0 = a0;
    pr.refine_b0 = b0;
    return launch_solve_refined(pr, B, fs->Lf32, fs->sl, fs->Uf32, X, st);
  }
  if (pen->two)
    return launch_solve2(pen->pt, pen->pb, B, fs->LfT, fs->slT, fs->UfT, fs->LfB, fs->slB, fs->UfB,
                         fs->Rinv, fs->E1, fs->E2, X, st);
  if (fs->sparse) return launch_solve_sparse(pen->pa, B, fs->sf, X, st);
  return launch_solve(pen->pa, B, fs->Lf, fs->sl, fs->Uf, X, st);
}

int stau_step(stau_pencils* pen, stau_state* s, double dt, void* stream) {
  if (!pen || !s || !s->X || !s->hist) return fail(STAU_EINVAL, "null argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(STAU_EINVAL, "dt must be positive");
  if (s->iteration > 0 && !(s->dt_prev > 0.0)) return fail(STAU_ESTATE, "dt_prev not set");
  if (s->head != 0 && s->head != 1) return fail(STAU_EINVAL, "head must be 0 or 1");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(pen->dom->d.device));
  double a0, a1, a2, b0, c1, c2;
  sbdf(s->iteration, dt, s->dt_prev, &a0, &a1, &a2, &b0, &c1, &c2);
  stau_pencils::FactorSlot* fs = nullptr;
  {
    int rc = factors_for(pen, a0, b0, st, &fs);
    if (rc) return rc;
  }
  const int cur = s->head ^ 1;
  const size_t hslot = (size_t)pen->dom->P * 2 * pen->pa.desc.ne * pen->dom->d.Nz;
  double2* hist = (double2*)s->hist;
  RhsArgs r{};
  r.mode = 1;
  r.c1 = c1;
  r.c2 = c2;
  r.a1 = a1;
  r.a2 = a2;
  r.has_hist = s->iteration > 0;
  r.Xprev = (const double2*)s->X;
  r.hist_cur = hist + cur * hslot;
  r.hist_old = hist + (cur ^ 1) * hslot;
  const bool mixed = pen->dom->d.precision == STAU_MIXED;
  HIP_TRY(explicit_term(pen, s->X, st, mixed));
  HIP_TRY(timed(pen, K_ZF, st, [&] {
    if (pen->dom->mm && !mixed) return launch_zf_mm(pen->xa, pen->H, pen->Bev, r, pen->dom->PLFzfrag, st);
    if (pen->dom->mm16 && mixed) return launch_zf_bf16(pen->xa, pen->H, pen->Bev, r, pen->dom->PLFz3, st);
    return launch_zf(pen->xa, pen->H, pen->Bev, r, st, mixed);
  }));
  HIP_TRY(timed(pen, K_SOLVE, st, [&] { return solve_launch(pen, fs, a0, b0, pen->Bev, s->X, st, mixed); }));
  s->head = cur;
  s->iteration += 1;
  s->dt_prev = dt;
  return STAU_OK;
}

namespace {
// IMEX Runge-Kutta tableaus with stages 0..s: H implicit (first row and
// column zero), A explicit (strictly lower triangular); the last stage is the
// step.  The (1,1,1), (2,2,2) and (4,4,3) schemes of Ascher, Ruuth & Spiteri.
struct RkTab {
  int s = 0;
  double A[5][5] = {}, H[5][5] = {};
};

bool rk_tableau(int scheme, RkTab* t) {
  *t = RkTab{};
  if (scheme == STAU_RK111) {
    t->s = 1;
    t->A[1][0] = 1.0;
    t->H[1][1] = 1.0;
  } else if (scheme == STAU_RK222) {
    const double g = 1.0 - 1.0 / std::sqrt(2.0), d = 1.0 - 1.0 / (2.0 * g);
    t->s = 2;
    t->A[1][0] = g;
    t->A[2][0] = d;
    t->A[2][1] = 1.0 - d;
    t->H[1][1] = g;
    t->H[2][1] = 1.0 - g;
    t->H[2][2] = g;
  } else if (scheme == STAU_RK443) {
    t->s = 4;
    const double A[5][5] = {{0, 0, 0, 0, 0},
                            {1.0 / 2, 0, 0, 0, 0},
                            {11.0 / 18, 1.0 / 18, 0, 0, 0},
                            {5.0 / 6, -5.0 / 6, 1.0 / 2, 0, 0},
                            {1.0 / 4, 7.0 / 4, 3.0 / 4, -7.0 / 4, 0}};
    const double H[5][5] = {{0, 0, 0, 0, 0},
                            {0, 1.0 / 2, 0, 0, 0},
                            {0, 1.0 / 6, 1.0 / 2, 0, 0},
                            {0, -1.0 / 2, 1.0 / 2, 1.0 / 2, 0},
                            {0, 3.0 / 2, -3.0 / 2, 1.0 / 2, 1.0 / 2}};
    std::memcpy(t->A, A, sizeof(A));
    std::memcpy(t->H, H, sizeof(H));
  } else {
    return false;
  }
  return true;
}
}  // namespace

int stau_step_rk(stau_pencils* pen, int scheme, double dt, void* X, void* stream) {
  if (!pen || !X) return fail(STAU_EINVAL, "null argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(STAU_EINVAL, "dt must be positive");
  RkTab tb;
  if (!rk_tableau(scheme, &tb)) return fail(STAU_EINVAL, "unknown Runge-Kutta scheme %d", scheme);
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(pen->dom->d.device));
  const int s = tb.s;
  const size_t field = (size_t)pen->dom->P * pen->pa.desc.ne * pen->dom->d.Nz;
  // F~ of stages 0..s-2, dt L~X of stages 1..s-2, M~X^{n,0}
  const int slots = (s - 1) + (s > 2 ? s - 2 : 0) + 1;
  if (pen->rk_slots < slots) {
    if (pen->rkbuf) {
      HIP_TRY(hipStreamSynchronize(st));
      HIP_TRY(hipFree(pen->rkbuf));
      pen->ws_bytes -= (int64_t)(pen->rk_slots * field * sizeof(double2));
      pen->rkbuf = nullptr;
      pen->rk_slots = 0;
    }
    if (hipMalloc(&pen->rkbuf, slots * field * sizeof(double2)) != hipSuccess)
      return fail(STAU_ENOMEM, "Runge-Kutta workspace allocation failed");
    pen->rk_slots = slots;
    pen->ws_bytes += (int64_t)(slots * field * sizeof(double2));
  }
  RhsArgs r{};
  r.mode = 2;
  r.Xprev = (const double2*)X;
  RkArgs& k = r.rk;
  k.dt = dt;
  int q = 0;
  for (int j = 0; j + 1 < s; ++j) k.F[j] = pen->rkbuf + (size_t)(q++) * field;
  for (int j = 1; j + 1 < s; ++j) k.K[j] = pen->rkbuf + (size_t)(q++) * field;
  k.MX0 = pen->rkbuf + (size_t)(q++) * field;
  k.Bprev = pen->Bev;
  const bool mixed = pen->dom->d.precision == STAU_MIXED;
  for (int i = 1; i <= s; ++i) {
    const double a0 = 1.0 / (dt * tb.H[i][i]), b0 = 1.0;
    stau_pencils::FactorSlot* fs = nullptr;
    {
      int rc = factors_for(pen, a0, b0, st, &fs);
      if (rc) return rc;
    }
    k.stage = i;
    k.last = i == s;
    k.scale = a0;
    k.hprev = i > 1 ? 1.0 / tb.H[i - 1][i - 1] : 0.0;
    for (int j = 0; j < kMaxRkStages; ++j) {
      k.A[j] = j < i ? tb.A[i][j] : 0.0;
      k.H[j] = j < i ? tb.H[i][j] : 0.0;
    }
    HIP_TRY(explicit_term(pen, X, st, mixed));
    HIP_TRY(timed(pen, K_ZF, st, [&] {
      if (pen->dom->mm && !mixed) return launch_zf_mm(pen->xa, pen->H, pen->Bev, r, pen->dom->PLFzfrag, st);
      if (pen->dom->mm16 && mixed) return launch_zf_bf16(pen->xa, pen->H, pen->Bev, r, pen->dom->PLFz3, st);
      return launch_zf(pen->xa, pen->H, pen->Bev, r, st, mixed);
    }));
    HIP_TRY(timed(pen, K_SOLVE, st, [&] { return solve_launch(pen, fs, a0, b0, pen->Bev, X, st, mixed); }));
  }
  return STAU_OK;
}

int stau_lbvp(stau_pencils* pen, const void* F, void* X, void* stream) {
  if (!pen || !F || !X) return fail(STAU_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(pen->dom->d.device));
  stau_pencils::FactorSlot* fs = nullptr;
  {
    int rc = factors_for(pen, 0.0, 1.0, st, &fs);
    if (rc) return rc;
  }
  HIP_TRY(launch_lbvp_rhs(pen->xa, F, pen->Bev, st));
  HIP_TRY(timed(pen, K_SOLVE, st, [&] { return solve_launch(pen, fs, 0.0, 1.0, pen->Bev, X, st, false); }));
  return STAU_OK;
}

int stau_evp(stau_pencils* pen, double tau, int nev, int ncv, int max_ops, double tol, double* sigma,
             double* resid, int32_t* nconv, int32_t* nops, void* X, void* stream) {
  if (!pen) return fail(STAU_EINVAL, "null argument");
  if (nev < 1 || nev > 16) return fail(STAU_EINVAL, "nev must be in [1, 16]");
  if (!sigma || !resid || !nconv) return fail(STAU_EINVAL, "null argument");
  if (!std::isfinite(tau)) return fail(STAU_EINVAL, "non-finite shift");
  if (ncv < nev + 2 || ncv > 32 || ncv > pen->pa.n)
    return fail(STAU_EINVAL, "ncv must be in [nev + 2, 32] and at most the pencil size");
  if (max_ops < ncv || max_ops > 1000000) return fail(STAU_EINVAL, "max_ops must be in [ncv, 1000000]");
  if (!(tol > 0.0 && tol < 1.0)) return fail(STAU_EINVAL, "tol must be in (0, 1)");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(pen->dom->d.device));
  PencilArgs pe = pen->pa;
  pe.lin = pen->par.b_top - pen->par.b_bottom;
  auto& f = pen->evp;
  if (!f.Lraw) {
    size_t bytes = 0;
    hipError_t e = alloc_slot(f, pe, &bytes);
    if (e != hipSuccess) return fail(STAU_ENOMEM, "factor allocation failed: %s", hipGetErrorString(e));
    pen->ws_bytes += (int64_t)bytes;
  }
  const size_t vbytes = (size_t)pe.P * (size_t)(ncv + 1) * (size_t)pe.n * sizeof(double);
  if (pen->evp_V_bytes < vbytes) {
    HIP_TRY(hipStreamSynchronize(st));
    if (pen->evp_V) (void)hipFree(pen->evp_V);
    pen->ws_bytes -= (int64_t)pen->evp_V_bytes;
    pen->evp_V = nullptr;
    pen->evp_V_bytes = 0;
    hipError_t e = hipMalloc((void**)&pen->evp_V, vbytes);
    if (e != hipSuccess) return fail(STAU_ENOMEM, "Krylov basis allocation failed: %s", hipGetErrorString(e));
    pen->evp_V_bytes = vbytes;
    pen->ws_bytes += (int64_t)vbytes;
  }
  if (!f.valid || f.a0 != tau) {
    f.valid = false;
    const int big = 0x7fffffff;
    HIP_TRY(hipMemcpyAsync(pen->sing, &big, sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(timed(pen, K_FACTOR, st, [&] { return launch_factor(pe, tau, 1.0, f.Lf, f.sl, f.Uf, pen->sing, st); }));
    int h = big;
    HIP_TRY(hipMemcpyAsync(&h, pen->sing, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h != big) {
      pen->last_sing = h;
      return fail(STAU_ESINGULAR, "zero or non-finite pivot in pencil %d (tau an eigenvalue?)", h);
    }
    f.valid = true;
    f.a0 = tau;
    f.b0 = 1.0;
  }
  const EvpOut o{(double2*)sigma, resid, (int*)nconv, (int*)nops, (double2*)X};
  HIP_TRY(timed(pen, K_SOLVE, st, [&] {
    return launch_evp(pe, tau, nev, ncv, max_ops, tol, f.Lf, f.sl, f.Uf, pen->evp_V, o, st);
  }));
  return STAU_OK;
}

int stau_initial_state(stau_pencils* pen, const double* b_grid, void* X, void* stream) {
  if (!pen || !b_grid || !X) return fail(STAU_EINVAL, "null argument");
  HIP_TRY(hipSetDevice(pen->dom->d.device));
  HIP_TRY(launch_initial_state(pen->xa1, b_grid, X, pen->scratch, (hipStream_t)stream));
  return STAU_OK;
}

}  // extern "C"

namespace {

// Fields of a variable mask (bit v: variable v of the state layout).
int vars_list(const stau_pencils* pen, uint32_t vars, FieldList* fl) {
  const int S = pen->pa.desc.S;
  if (vars == 0 || (vars >> S) != 0)
    return fail(STAU_EINVAL, "vars 0x%x must be a non-empty mask of the %d state variables", vars, S);
  *fl = FieldList{};
  for (int v = 0; v < S; ++v)
    if (vars & (1u << v)) {
      fl->var[fl->nf] = v;
      fl->deriv[fl->nf] = 0;
      ++fl->nf;
    }
  return STAU_OK;
}

// Transform description and grid sizes of a grid scale (1 or 3/2).
int grid_args(const stau_pencils* pen, double scale, XformArgs* xa, int* Lg, int* Ngy, int* Mg) {
  if (scale == 1.0)
    *xa = pen->xa1;
  else if (scale == 1.5)
    *xa = pen->xa;
  else
    return fail(STAU_EINVAL, "scale must be 1 or 1.5");
  *Lg = xa->L;
  *Ngy = xa->dim == 3 ? xa->Ngy : 1;
  *Mg = xa->M;
  if (!xgrid_supported(*Lg, *Mg)) return fail(STAU_EUNSUPPORTED, "grid of %d x points unsupported", *Lg);
  return STAU_OK;
}

}  // namespace

extern "C" {

int stau_coeff_to_grid(stau_pencils* pen, const void* X, uint32_t vars, double scale, double* grid,
                       void* stream) {
  if (!pen || !X || !grid) return fail(STAU_EINVAL, "null argument");
  FieldList fl;
  XformArgs xa;
  int Lg, Ngy, Mg, rc;
  if ((rc = vars_list(pen, vars, &fl)) || (rc = grid_args(pen, scale, &xa, &Lg, &Ngy, &Mg))) return rc;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(pen->dom->d.device));
  HIP_TRY(launch_zb(xa, fl, X, pen->G, st));
  const void* rows = pen->G;
  if (xa.dim == 3) {
    HIP_TRY(launch_ypass(xa, +1, fl.nf, pen->G, pen->G2, st));
    rows = pen->G2;
  }
  HIP_TRY(launch_xgrid(xa, +1, fl.nf, Lg, Ngy, Mg, xa.twx, rows, grid, 1.0, 1.0, st));
  return STAU_OK;
}

int stau_grid_to_coeff(stau_pencils* pen, const double* grid, uint32_t vars, double scale, void* X,
                       void* stream) {
  if (!pen || !X || !grid) return fail(STAU_EINVAL, "null argument");
  FieldList fl;
  XformArgs xa;
  int Lg, Ngy, Mg, rc;
  if ((rc = vars_list(pen, vars, &fl)) || (rc = grid_args(pen, scale, &xa, &Lg, &Ngy, &Mg))) return rc;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(pen->dom->d.device));
  const bool d3 = xa.dim == 3;
  // x analysis to spectral rows, (y analysis,) z analysis to F[P][nf][N]
  double2* rows = d3 ? pen->G2 : pen->G;
  HIP_TRY(launch_xgrid(xa, -1, fl.nf, Lg, Ngy, Mg, xa.twx, grid, rows, 1.0 / Lg, 1.0 / Lg, st));
  if (d3) HIP_TRY(launch_ypass(xa, -1, fl.nf, pen->G2, pen->G, st));
  double2* F = d3 ? pen->G2 : pen->Gb;
  XformArgs az = xa;
  az.ne = fl.nf;
  RhsArgs r{};
  r.mode = 0;
  HIP_TRY(launch_zf(az, pen->G, F, r, st));
  HIP_TRY(launch_put_vars(xa.P, xa.S, xa.N, fl, F, X, st));
  return STAU_OK;
}

int stau_coeff_to_grid_adjoint(stau_pencils* pen, const double* grid_bar, uint32_t vars, double scale,
                               void* X_bar, void* stream) {
  if (!pen || !X_bar || !grid_bar) return fail(STAU_EINVAL, "null argument");
  FieldList fl;
  XformArgs xa;
  int Lg, Ngy, Mg, rc;
  if ((rc = vars_list(pen, vars, &fl)) || (rc = grid_args(pen, scale, &xa, &Lg, &Ngy, &Mg))) return rc;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(pen->dom->d.device));
  const bool d3 = xa.dim == 3;
  HIP_TRY(launch_zero_vars(xa.P, xa.S, xa.N, fl, X_bar, st));
  // adjoint of the x synthesis: analysis with weights 1 (k = 0) and 2
  double2* rows = d3 ? pen->G2 : pen->G;
  HIP_TRY(launch_xgrid(xa, -1, fl.nf, Lg, Ngy, Mg, xa.twx, grid_bar, rows, 1.0, 2.0, st));
  // adjoint of the y synthesis: the analysis without the 1 / Ngy
  if (d3) HIP_TRY(launch_ypass(xa, -1, fl.nf, pen->G2, pen->G, st, false, 1.0));
  // adjoint of the z synthesis, accumulated into the zeroed variables
  AccList al{};
  al.nt = fl.nf;
  for (int f = 0; f < fl.nf; ++f) {
    al.target[f] = fl.var[f];
    al.nsrc[f] = 1;
    al.src[f][0] = f;
    al.src[f][1] = -1;
  }
  HIP_TRY(launch_zadj(xa, al, pen->G, X_bar, st));
  return STAU_OK;
}

int stau_grid_to_coeff_adjoint(stau_pencils* pen, const void* X_bar, uint32_t vars, double scale,
                               double* grid_bar, void* stream) {
  if (!pen || !X_bar || !grid_bar) return fail(STAU_EINVAL, "null argument");
  FieldList fl;
  XformArgs xa;
  int Lg, Ngy, Mg, rc;
  if ((rc = vars_list(pen, vars, &fl)) || (rc = grid_args(pen, scale, &xa, &Lg, &Ngy, &Mg))) return rc;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(pen->dom->d.device));
  // adjoint of the z analysis: synthesis of the coefficients weighted by
  // (2 - delta_n0) / Mg
  fl.wmode = 1;
  HIP_TRY(launch_zb(xa, fl, X_bar, pen->G, st));
  const void* rows = pen->G;
  if (xa.dim == 3) {
    // adjoint of the y analysis: the synthesis scaled by 1 / Ngy
    HIP_TRY(launch_ypass(xa, +1, fl.nf, pen->G, pen->G2, st, false, 1.0 / Ngy));
    rows = pen->G2;
  }
  // adjoint of the x analysis: synthesis with weights 1 / Lg (k = 0) and 1 / (2 Lg)
  HIP_TRY(launch_xgrid(xa, +1, fl.nf, Lg, Ngy, Mg, xa.twx, rows, grid_bar, 1.0 / Lg, 0.5 / Lg, st));
  return STAU_OK;
}

int stau_nonlinear(stau_pencils* pen, const void* X, void* F, void* stream) {
  if (!pen || !X || !F) return fail(STAU_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(pen->dom->d.device));
  RhsArgs r{};
  r.mode = 0;
  HIP_TRY(explicit_term(pen, X, st, false));
  if (pen->dom->mm)
    HIP_TRY(launch_zf_mm(pen->xa, pen->H, F, r, pen->dom->Fzfrag, st));
  else
    HIP_TRY(launch_zf(pen->xa, pen->H, F, r, st));
  return STAU_OK;
}

int stau_solve(stau_pencils* pen, const void* B_ev, void* X, void* stream) {
  if (!pen || !B_ev || !X) return fail(STAU_EINVAL, "null argument");
  if (!pen->has_last) return fail(STAU_ESTATE, "stau_solve before a successful stau_factor");
  HIP_TRY(hipSetDevice(pen->dom->d.device));
  // the slot stau_factor filled may have been refactored since for another
  // operator (the step's and the boundary value solve's cache is shared)
  stau_pencils::FactorSlot* f = nullptr;
  {
    int rc = factors_for(pen, pen->last_a0, pen->last_b0, (hipStream_t)stream, &f);
    if (rc) return rc;
  }
  if (pen->two)
    HIP_TRY(launch_solve2(pen->pt, pen->pb, B_ev, f->LfT, f->slT, f->UfT, f->LfB, f->slB, f->UfB, f->Rinv,
                          f->E1, f->E2, X, (hipStream_t)stream));
  else
    if (f->sparse)
      HIP_TRY(launch_solve_sparse(pen->pa, B_ev, f->sf, X, (hipStream_t)stream));
    else
      HIP_TRY(launch_solve(pen->pa, B_ev, f->Lf, f->sl, f->Uf, X, (hipStream_t)stream));
  return STAU_OK;
}

int stau_adjoint_step(stau_pencils* pen, const void* X_prev, int64_t iteration, double dt,
                      double dt_prev, stau_adjstate* adj, void* stream) {
  if (!pen || !X_prev || !adj || !adj->Xbar || !adj->hbar) return fail(STAU_EINVAL, "null argument");
  if (pen->dom->d.dim != 2) return fail(STAU_EUNSUPPORTED, "the adjoint is built for 2-D domains");
  if (!pen->adj_ok) return fail(STAU_EUNSUPPORTED, "transposed band too wide for the adjoint (n_gamma)");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(STAU_EINVAL, "dt must be positive");
  if (iteration < 0 || (iteration > 0 && !(dt_prev > 0.0)))
    return fail(STAU_EINVAL, "iteration / dt_prev inconsistent");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(pen->dom->d.device));
  double a0, a1, a2, b0, c1, c2;
  sbdf(iteration, dt, dt_prev, &a0, &a1, &a2, &b0, &c1, &c2);
  stau_pencils::FactorSlot* fs = nullptr;
  {
    int rc = factors_for(pen, a0, b0, st, &fs, true);
    if (rc) return rc;
  }
  AdjRhsArgs r{};
  r.c1 = c1;
  r.c2 = c2;
  r.a1 = a1;
  r.a2 = a2;
  r.hbar = (double2*)adj->hbar;
  r.Fbar = pen->Bev;
  // mixed precision: FP32 adjoint transforms; the transposed solve is FP64
  // (FP32 sweeps with an FP64 residual and a correction sweep measured slower:
  // 512x128 adjoint step 260 -> 150 us, 4096x64 303 -> 273 us), and X_bar,
  // F_bar and the history stay FP64
  const bool mixed = pen->dom->d.precision == STAU_MIXED;
  // 3. (forward grid fields at X^{n-1}) needs only X_prev: it runs on the side
  // stream, overlapping steps 1 and 2, which leave pen->G alone
  if (!pen->side) {
    HIP_TRY(hipStreamCreateWithFlags(&pen->side, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&pen->ev_fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&pen->ev_join, hipEventDisableTiming));
  }
  HIP_TRY(hipEventRecord(pen->ev_fork, st));
  HIP_TRY(hipStreamWaitEvent(pen->side, pen->ev_fork, 0));
  HIP_TRY(launch_zb(pen->xa, pen->fl_adj, X_prev, pen->G, pen->side, mixed));
  HIP_TRY(hipEventRecord(pen->ev_join, pen->side));
  // 1. transposed pencil solve + multistep history adjoints
  if (pen->twoT)
    HIP_TRY(launch_solve2T(pen->ptT, pen->pbT, adj->Xbar, fs->LfT, fs->slT, fs->UfT, fs->LfB, fs->slB,
                           fs->UfB, fs->Rinv, fs->E1, fs->E2, adj->Xbar, r, st));
  else
    HIP_TRY(launch_solveT(pen->paT, adj->Xbar, fs->Lf, fs->sl, fs->Uf, adj->Xbar, r, st));
  // 2. adjoint of the forward z transform: H_bar = W^T F_bar
  FieldList fe{};
  fe.nf = pen->pa.desc.ne;
  for (int e = 0; e < fe.nf; ++e) fe.var[e] = e;
  fe.src_S = pen->pa.desc.ne;
  fe.wmode = 1;
  HIP_TRY(launch_zb(pen->xa, fe, pen->Bev, pen->H, st, mixed));
  // (join step 3)
  HIP_TRY(hipStreamWaitEvent(st, pen->ev_join, 0));
  // 4. adjoint x pass
  HIP_TRY(launch_xpass_adj(pen->xa, pen->G, pen->H, pen->Gb, st, mixed));
  // 5. adjoint of the backward z transform, accumulated into X_bar
  HIP_TRY(launch_zadj(pen->xa, pen->acc, pen->Gb, adj->Xbar, st, mixed));
  return STAU_OK;
}

int stau_kinetic_energy_adjoint(stau_pencils* pen, const void* X, void* Xbar, void* stream) {
  if (!pen || !X || !Xbar) return fail(STAU_EINVAL, "null argument");
  if (pen->dom->d.dim != 2) return fail(STAU_EUNSUPPORTED, "the adjoint is built for 2-D domains");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(pen->dom->d.device));
  double2* ebar = (double2*)pen->scratch;
  HIP_TRY(launch_ke_adjoint(pen->xa, X, pen->G, pen->Gb, pen->wvec, ebar, Xbar, st));
  return STAU_OK;
}

int stau_initial_state_adjoint(stau_pencils* pen, const void* Xbar, double* b_grid_bar,
                               void* stream) {
  if (!pen || !Xbar || !b_grid_bar) return fail(STAU_EINVAL, "null argument");
  if (pen->dom->d.dim != 2) return fail(STAU_EUNSUPPORTED, "the adjoint is built for 2-D domains");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(pen->dom->d.device));
  HIP_TRY(launch_initial_state_adjoint(pen->xa1, Xbar, b_grid_bar, pen->scratch, st));
  return STAU_OK;
}

__global__ void nonfinite_kernel(const double* x, size_t n, int* flag) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  for (; i < n; i += (size_t)gridDim.x * blockDim.x)
    if (!isfinite(x[i])) {
      atomicOr(flag, 1);
      return;
    }
}

int stau_check(stau_pencils* pen, const void* X, void* stream) {
  if (!pen || !X) return fail(STAU_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(pen->dom->d.device));
  const int zero = 0;
  HIP_TRY(hipMemcpyAsync(pen->flag, &zero, sizeof(int), hipMemcpyHostToDevice, st));
  const size_t nd = (size_t)pen->dom->P * pen->pa.desc.S * pen->dom->d.Nz * 2;
  hipLaunchKernelGGL(nonfinite_kernel, dim3(1024), dim3(256), 0, st, (const double*)X, nd,
                     pen->flag);
  HIP_TRY(hipGetLastError());
  int h = 0;
  HIP_TRY(hipMemcpyAsync(&h, pen->flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (h) return fail(STAU_ENONFINITE, "state holds non-finite values");
#ifdef STAU_CHECK_BOUNDS
  unsigned bits = 0;
  HIP_TRY(hipMemcpy(&bits, pen->check, sizeof(unsigned), hipMemcpyDeviceToHost));
  if (bits)
    return fail(STAU_EBOUNDS, "index check failed since the pencils were built (bits 0x%x: 1 pivot offset, "
                "2 sparse record size, 4 forward-window slot, 8 record rank)", bits);
#endif
  return STAU_OK;
}

int stau_kinetic_energy_noalloc(stau_pencils* pen, const void* X, double* out, void* stream) {
  if (!pen || !X || !out) return fail(STAU_EINVAL, "null argument");
  const int dev = pen->dom->d.device;
  HIP_TRY(hipSetDevice(dev));
  void* sp = nullptr;
  {
    const int rc = scratch_address(dev, &sp);
    if (rc) return rc;
  }
  // the same kernels as stau_kinetic_energy, with every intermediate in the
  // device's scratch array: G [nf][M][P], G2 [nf][M][Ngy][Px] (3-D), rowmean
  // [M Ngy]; the result goes to the caller's device double.  Every entry is
  // written before it is read, so nothing needs clearing between calls.
  const XformArgs& a = pen->xa;
  const size_t nf = a.dim == 2 ? 2 : 3, R = (size_t)a.M * (a.dim == 3 ? a.Ngy : 1);
  const size_t bG = nf * a.M * a.P * sizeof(double2);
  const size_t bG2 = a.dim == 3 ? nf * R * a.Px * sizeof(double2) : 0;
  const size_t bR = (R * sizeof(double) + 255) / 256 * 256;
  const size_t need = bG + bG2 + bR;
  if (need > kNoAllocBytes)
    return fail(STAU_EUNSUPPORTED, "no-allocation kinetic energy needs %zu bytes of scratch (limit %zu)",
                need, kNoAllocBytes);
  char* base = (char*)sp;
  void* G = base;
  void* G2 = a.dim == 3 ? base + bG : nullptr;
  double* rowmean = (double*)(base + bG + bG2);
  HIP_TRY(launch_ke(a, X, G, G2, rowmean, out, (hipStream_t)stream));
  return STAU_OK;
}

int stau_kinetic_energy(stau_pencils* pen, const void* X, double* out, void* stream) {
  if (!pen || !X || !out) return fail(STAU_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(pen->dom->d.device));
  double* rowmean = (double*)pen->scratch;
  double* dout = rowmean + (size_t)pen->xa.M * pen->dom->Ngy;
  HIP_TRY(launch_ke(pen->xa, X, pen->G, pen->G2, rowmean, dout, st));
  HIP_TRY(hipMemcpyAsync(out, dout, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return STAU_OK;
}

}  // extern "C"
