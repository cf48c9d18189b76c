// sieve.hip -- host runtime and C ABI of the MI355X segmented odd-only sieve.
// The entry points are declared and documented in include/sieve.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "sieve.h"
#include "kernels.inc"
#include "logsieve.inc"

namespace {

thread_local int g_last_hip = 0;

struct DevBuf;
// Dry run: while set, DevBuf::ensure records the size it would grow to instead of
// allocating, and no kernel, copy or event is enqueued (a pure host planning pass
// that gives the exact device bytes of a call).
struct DryRun {
  std::vector<std::pair<const DevBuf*, size_t>> want;
  void note(const DevBuf* b, size_t n) {
    for (auto& w : want)
      if (w.first == b) { w.second = std::max(w.second, n); return; }
    want.emplace_back(b, n);
  }
};
thread_local DryRun* g_dry = nullptr;
// The stream of the call in progress on this thread: a growing buffer waits for
// the work enqueued on it (the context's earlier calls are ordered before it)
// before the old memory is released.
thread_local hipStream_t g_call_stream = nullptr;
thread_local bool g_in_call = false;

#define HIPCHK(expr)                                   \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) {                            \
      g_last_hip = (int)e_;                            \
      return SIEVE_E_HIP;                              \
    }                                                  \
  } while (0)

#define STCHK(expr)                 \
  do {                              \
    int s_ = (expr);                \
    if (s_ != SIEVE_OK) return s_;  \
  } while (0)

constexpr uint64_t kLaunchBits = sv::kWinBits;  // offsets of one launch window fit 32 bits
constexpr uint32_t kGenTile = 20;             // largest tile of the prime generator
constexpr uint32_t kBatchRunMax = 16;         // most consecutive tiles per batch work item
constexpr uint32_t kAutoRangeBins = 1024;      // chunks with this many bins or more use two bin ranges by default
constexpr double kHitsPerGroup = 16384.0;      // fewest expected hits per bucket-fill workgroup
constexpr uint32_t kMaxCountBins = 32768;      // bins of one count job (its LDS histogram: 128 KB)

// Grow-only device buffer.  A fixed buffer is a slice of the library's static
// scratch array: it never grows, and a request beyond its size is an error.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool fixed = false;
  int ensure(size_t n) {
    if (g_dry) { g_dry->note(this, std::max<size_t>(n, 256)); return SIEVE_OK; }
    if (n <= bytes) return SIEVE_OK;
    if (fixed) return SIEVE_E_SCRATCH;
    if (p) {
      // earlier users must be done before the memory is released: the kernels of
      // this call and of the owner's earlier calls, all ordered on the call's stream
      hipError_t e = g_in_call ? hipStreamSynchronize(g_call_stream) : hipDeviceSynchronize();
      if (e != hipSuccess) { g_last_hip = (int)e; return SIEVE_E_HIP; }
      (void)hipFree(p);
      p = nullptr;
      bytes = 0;
    }
    size_t want = std::max<size_t>(n, 256);
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) { g_last_hip = (int)e; p = nullptr; return SIEVE_E_NOMEM; }
    bytes = want;
    return SIEVE_OK;
  }
  void release() {
    if (fixed) return;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename T> T* as() const { return reinterpret_cast<T*>(p); }
};

// Rosser-Schoenfeld style bounds (all primes, so they also bound the odd ones).
uint64_t pi_upper(uint64_t x) {
  if (x < 100) return 26;
  double v = 1.25506 * (double)x / std::log((double)x);
  return (uint64_t)v + 64;
}
// Upper bound on sum of 1/p for lo <= p <= hi (lo >= 286): loglog(hi) - loglog(lo) + 1/ln^2(lo).
double recip_sum_upper(double lo, double hi) {
  if (hi < lo) return 0.0;
  lo = std::max(lo, 286.0);
  double l1 = std::log(lo);
  return std::log(std::log(std::max(hi, lo))) - std::log(l1) + 1.0 / (l1 * l1);
}

uint64_t isqrt_u64(uint64_t x) {
  uint64_t r = (uint64_t)std::sqrt((double)x);
  while (r > 0 && (unsigned __int128)r * r > x) --r;
  while ((unsigned __int128)(r + 1) * (r + 1) <= x) ++r;
  return r;
}

struct Resolved {
  uint32_t L, Mlog, Wlog, Blog, binslog, groups, b, R, sparse;
};

int resolve_tune(uint32_t l, const sieve_tune* t, Resolved* r) {
  sieve_tune z;
  memset(&z, 0, sizeof z);
  if (!t) t = &z;
  r->L = t->tile_log2 ? t->tile_log2 : std::min<uint32_t>(20, std::max<uint32_t>(15, l));
  if (r->L < 13 || r->L > 20 || r->L > l + 10) return SIEVE_E_ARG;  // per-tile count slots fit LDS
  r->Mlog = t->medium_log2 ? t->medium_log2 : r->L;
  if (r->Mlog + 4 < r->L || r->Mlog > r->L + 1) return SIEVE_E_ARG;
  r->Wlog = t->wave_log2 ? t->wave_log2 : 9;
  r->Blog = t->wheel_log2 ? t->wheel_log2 : std::max<uint32_t>(r->Wlog, std::min<uint32_t>(r->L - 7, r->Mlog));
  if (r->Wlog < 9 || r->Wlog > r->Blog || r->Blog > r->Mlog) return SIEVE_E_ARG;
  r->b = t->bin_log2 ? t->bin_log2 : r->L;
  if (r->b < std::min<uint32_t>(r->L, 16) || r->b > r->L) return SIEVE_E_ARG;
  r->binslog = t->bins_log2 ? t->bins_log2 : std::min<uint32_t>(15, 31 - r->b);
  if (r->binslog < 8 || r->binslog > 15) return SIEVE_E_ARG;
  r->R = t->ranges;                              // 0: chosen per chunk
  if (r->R != 0 && r->R != 1 && r->R != 2 && r->R != 4 && r->R != 8) return SIEVE_E_ARG;
  r->groups = t->groups ? t->groups : 2048;
  if (r->groups < 64 || r->groups > 4096) return SIEVE_E_ARG;
  if (r->R) r->groups -= r->groups % r->R;
  r->sparse = t->sparse;
  if (r->sparse > 2) return SIEVE_E_ARG;
  return SIEVE_OK;
}

int check_interval(uint32_t l, uint64_t f, uint64_t n, uint64_t B, uint64_t* F, uint64_t* NB) {
  if (l < 5 || l > 20 || n == 0) return SIEVE_E_ARG;
  if (B < 3 || B >= (1ull << 32)) return SIEVE_E_BOUND;
  unsigned __int128 FF = (unsigned __int128)f << l, NN = (unsigned __int128)n << l;
  unsigned __int128 v = 2 * (FF + NN);
  if (v >> 64) return SIEVE_E_RANGE;
  *F = (uint64_t)FF;
  *NB = (uint64_t)NN;
  return SIEVE_OK;
}

}  // namespace

struct sieve_primes {
  int device = 0;
  uint64_t B = 0;
  uint64_t count = 0;
  DevBuf P, cnt;
};

struct KernelTime {
  double ms = 0;
  uint64_t n = 0;
};

struct sieve_ctx {
  std::mutex mu;
  int device = 0;
  uint32_t ncu = 0;                 // compute units of the device
  hipStream_t last_stream = nullptr;
  bool has_last = false;
  hipEvent_t done = nullptr;
  // scratch
  DevBuf plan, Q0, OFF, HG, PS, bstart, bucket, err, gen_S, gen_blk, mb_sink;
  // batch scratch and the host copies of its tables
  DevBuf b_req, b_blk, b_seg0, b_tcnt, b_queue, b_items, jobs, blk2job, cjobs, cblk2job, thr;
  DevBuf gb_best, gb_k;   // Goldbach check: packed per-segment maxima, prime count
  DevBuf wsl;             // intervals beyond 2^64: a sieved slice of the primes above 2^32
  DevBuf logpat;          // log-add sieve: weights of 3..13 over one period
  DevBuf spE, spH;        // sparse large primes: sorted hits per collecting workgroup, bin headers
  DevBuf wH, wHc, wE, wHd;  // primes above 2^32: hit slots and counts, sorted regions, bin headers
  std::vector<sv::BatchReq> h_req;
  std::vector<uint2> h_blk, h_items;
  std::vector<uint32_t> h_seg0;
  std::vector<sv::BucketJob> h_jobs, h_cjobs;           // scatter jobs (bin ranges), count jobs (whole chunks)
  std::vector<uint32_t> h_blk2job, h_cblk2job, h_thr;
  // pinned staging for host-to-device table copies; reused only after the
  // previous call's copies have completed (pin_ev)
  void* pin = nullptr;
  size_t pin_bytes = 0, pin_used = 0;
  hipEvent_t pin_ev = nullptr;
  bool pin_pending = false;
  DevBuf pat[32], xpat;
  uint32_t pat_words[32] = {0};
  bool xpat_ready = false, err_ready = false;   // built / cleared on the device
  sieve_primes own;  // table built by sieve_init / sieve_ctx_sieve
  // timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  struct Pending { std::string name; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::map<std::string, KernelTime> times;
  // every device buffer the context owns
  template <typename F>
  void each_buf(F&& f) {
    DevBuf* bufs[] = {&plan, &Q0, &OFF, &HG, &PS, &bstart, &bucket, &err, &gen_S, &gen_blk, &mb_sink,
                      &b_req, &b_blk, &b_seg0, &b_tcnt, &b_queue, &b_items, &jobs, &blk2job, &cjobs, &cblk2job, &thr,
                      &own.P, &own.cnt, &xpat, &gb_best, &gb_k, &wsl, &logpat, &spE, &spH,
                      &wH, &wHc, &wE, &wHd};
    for (DevBuf* b : bufs) f(*b);
    for (auto& b : pat) f(b);
  }
  ~sieve_ctx();
};

sieve_ctx::~sieve_ctx() {
  if (has_last) (void)hipStreamSynchronize(last_stream);
  each_buf([](DevBuf& b) { b.release(); });
  for (auto& e : ev_pool) (void)hipEventDestroy(e);
  for (auto& p : pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
  if (done) (void)hipEventDestroy(done);
  if (pin_pending && pin_ev) (void)hipEventSynchronize(pin_ev);
  if (pin) (void)hipHostFree(pin);
  if (pin_ev) (void)hipEventDestroy(pin_ev);
}

namespace {

hipEvent_t take_event(sieve_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Launch wrapper: records an event pair around the kernel when timing is on.
template <typename F>
int launch(sieve_ctx* c, const char* name, hipStream_t s, F&& f) {
  if (g_dry) return SIEVE_OK;
  hipEvent_t a = nullptr, b = nullptr;
  if (c->timing) {
    a = take_event(c);
    b = take_event(c);
    if (a && b) HIPCHK(hipEventRecord(a, s));
  }
  f();
  HIPCHK(hipGetLastError());
  if (c->timing && a && b) {
    HIPCHK(hipEventRecord(b, s));
    c->pending.push_back({name, a, b});
  }
  return SIEVE_OK;
}

int collect_times(sieve_ctx* c) {
  for (auto& p : c->pending) {
    HIPCHK(hipEventSynchronize(p.b));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
    auto& kt = c->times[p.name];
    kt.ms += ms;
    kt.n += 1;
    c->ev_pool.push_back(p.a);
    c->ev_pool.push_back(p.b);
  }
  c->pending.clear();
  return SIEVE_OK;
}

// Pinned staging: pin_begin waits for the previous call's copies, reserves
// `total` bytes; upload copies a host table into it and enqueues the copy;
// pin_end records the event that guards the next reuse.
int pin_begin(sieve_ctx* c, size_t total) {
  if (g_dry) return SIEVE_OK;
  if (c->pin_pending) {
    HIPCHK(hipEventSynchronize(c->pin_ev));
    c->pin_pending = false;
  }
  c->pin_used = 0;
  if (total > c->pin_bytes) {
    if (c->pin) (void)hipHostFree(c->pin);
    c->pin = nullptr;
    c->pin_bytes = 0;
    const size_t want = std::max<size_t>(total * 2, 1 << 16);
    HIPCHK(hipHostMalloc(&c->pin, want, hipHostMallocDefault));
    c->pin_bytes = want;
  }
  if (!c->pin_ev) HIPCHK(hipEventCreateWithFlags(&c->pin_ev, hipEventDisableTiming));
  return SIEVE_OK;
}
int upload(sieve_ctx* c, hipStream_t s, void* dst, const void* src, size_t n) {
  if (!n || g_dry) return SIEVE_OK;
  if (c->pin_used + n > c->pin_bytes) return SIEVE_E_ARG;
  char* p = static_cast<char*>(c->pin) + c->pin_used;
  memcpy(p, src, n);
  HIPCHK(hipMemcpyAsync(dst, p, n, hipMemcpyHostToDevice, s));
  c->pin_used += (n + 255) & ~size_t(255);
  return SIEVE_OK;
}
int pin_end(sieve_ctx* c, hipStream_t s) {
  if (g_dry) return SIEVE_OK;
  if (c->pin_used) {
    HIPCHK(hipEventRecord(c->pin_ev, s));
    c->pin_pending = true;
  }
  return SIEVE_OK;
}
size_t pad256(size_t n) { return (n + 255) & ~size_t(255); }

// Thresholds that split the large primes lo_p <= p <= B of a job into GR slices of
// equal estimated work: span/p hits per prime in the job's span of bits plus a
// per-prime cost of four hits (prime density 1/ln x; Mertens for the hit sum).
void work_thresholds(double lo_p, double B, double span, uint32_t GR, uint32_t* thr) {
  thr[0] = 0;
  if (GR <= 1) return;
  const int NS = 512;
  std::vector<double> xs(NS + 1), W(NS + 1, 0.0);
  const double r = std::log(std::max(B, lo_p + 1.0) / lo_p);
  for (int i = 0; i <= NS; ++i) xs[i] = lo_p * std::exp(r * i / NS);
  for (int i = 1; i <= NS; ++i) {
    const double a = xs[i - 1], b = xs[i], mid = 0.5 * (a + b);
    const double count = (b - a) / std::log(mid);
    const double hits = span * (std::log(std::log(b)) - std::log(std::log(a)));
    W[i] = W[i - 1] + hits + 2.0 * count;
  }
  int i = 1;
  for (uint32_t q = 1; q < GR; ++q) {
    const double target = W[NS] * q / GR;
    while (i < NS && W[i] < target) ++i;
    const double f = (W[i] > W[i - 1]) ? (target - W[i - 1]) / (W[i] - W[i - 1]) : 0.0;
    const double x = xs[i - 1] + f * (xs[i] - xs[i - 1]);
    thr[q] = (uint32_t)std::min(std::max(x, (double)thr[q - 1]), 4294967295.0);
  }
}

// Dynamic LDS of one scatter launch whose jobs have at most max_rbins bins: stages of
// kMinStageBytes per bin at least and up to kMaxStageBytes, plus the counters.  The
// scatter is latency bound, so when the smallest stages fit in kScatterLdsPair the
// launch stays within it and two workgroups (32 waves) share a CU.
constexpr uint32_t kScatterLds = 152 * 1024;       // 2048 bins * (64 + 12) bytes
constexpr uint32_t kScatterLdsPair = 72 * 1024;    // (160 KB - 2 * 8 KB static) / 2
uint32_t scatter_lds(uint32_t max_rbins) {
  const uint64_t per = sv::kStageWords * 4;
  const uint64_t lo = (uint64_t)max_rbins * (per + sv::kMinStageBytes);
  const uint64_t lim = lo <= kScatterLdsPair ? kScatterLdsPair : kScatterLds;
  const uint64_t hi = std::min<uint64_t>((uint64_t)max_rbins * (per + sv::kMaxStageBytes), lim);
  return (uint32_t)std::max(lo, hi);
}

// log2 of the stage entries per bin of a job with rbins bins in a launch of lds bytes
// (the largest power of two that fits, at most 2^cap, at least kMinStageBytes).
uint32_t stage_log2(uint32_t lds, uint32_t rbins, uint32_t esz, uint32_t cap = 31) {
  const uint32_t per = std::min<uint32_t>(lds / rbins - sv::kStageWords * 4, sv::kMaxStageBytes) / esz;
  uint32_t l2 = 0;
  while ((2u << l2) <= per) ++l2;
  uint32_t lo = 0;
  while ((1u << lo) * esz < sv::kMinStageBytes) ++lo;
  return std::max(lo, std::min(l2, cap));
}

// Sets the stage size of jobs [j0, j1) for one scatter launch and returns the
// padding the group-rounded regions can add to the bucket (entries).
uint64_t set_stages(std::vector<sv::BucketJob>& jobs, size_t j0, size_t j1, uint32_t esz, uint32_t* lds_out) {
  uint32_t max_rbins = 1;
  for (size_t k = j0; k < j1; ++k) max_rbins = std::max(max_rbins, jobs[k].rbins);
  const uint32_t lds = scatter_lds(max_rbins);
  uint64_t pad = 0;
  for (size_t k = j0; k < j1; ++k) {
    jobs[k].sbl = stage_log2(lds, jobs[k].rbins, esz, jobs[k].sbl);
    pad += (uint64_t)jobs[k].GR * jobs[k].rbins * (sv::kRegionBytes / esz - 1);
  }
  if (lds_out) *lds_out = lds;
  return pad;
}

int set_lds_limits() {
  static std::once_flag once;
  static int rc = SIEVE_OK;
  std::call_once(once, [] {
    // 160 KB per CU minus the bucket kernels' static LDS (kLoad primes and offsets,
    // 8 KB); the scatter's stages and counters use at most 152 KB
    const int lim = kScatterLds;
    const void* fns[] = {(const void*)sv::k_bucket_count2, (const void*)sv::k_bucket_scatter2<uint16_t>,
                         (const void*)sv::k_bucket_scatter2<uint32_t>, (const void*)sv::k_bucket_scatter2<uint32_t, true>,
                         (const void*)sv::k_sparse_apply};
    for (const void* f : fns)
      if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess) rc = SIEVE_E_HIP;
  });
  return rc;
}

// Pattern of the primes 3..13 that are <= B (Section 3.1's small primes, applied
// as one periodic mask instead of per-prime masks).
int get_pattern(sieve_ctx* c, uint64_t B, hipStream_t s, const uint32_t** pat, uint32_t* per,
                uint32_t* words, uint32_t* mask) {
  static const uint32_t small[5] = {3, 5, 7, 11, 13};
  uint32_t m = 0, P = 1;
  sv::PatPrimes pp;
  memset(&pp, 0, sizeof pp);
  for (int i = 0; i < 5; ++i)
    if (small[i] <= B) { m |= 1u << i; P *= small[i]; pp.p[pp.n++] = small[i]; }
  // one period plus the wrap-around of a wave block starting anywhere in it, in
  // whole 16-byte groups
  const uint32_t nw = ((P + sv::kPatWrapBits + 31) / 32 + 3) & ~3u;
  if (!c->pat_words[m]) {
    STCHK(c->pat[m].ensure((size_t)nw * 4));
    STCHK(launch(c, "k_pattern", s, [&] {
      sv::k_pattern<<<(nw + 255) / 256, 256, 0, s>>>(c->pat[m].as<uint32_t>(), P, pp, nw);
    }));
    if (!g_dry) c->pat_words[m] = nw;
  }
  *pat = c->pat[m].as<uint32_t>();
  *per = P;
  *words = nw;
  *mask = m;
  return SIEVE_OK;
}

// The patterns of 17*19*23, 29*31*37 and 41*43*47 (built once per context).
int get_xpattern(sieve_ctx* c, hipStream_t s, const uint32_t** xpat) {
  if (!c->xpat_ready) {
    STCHK(c->xpat.ensure((size_t)sv::kXWordsAll * 4));
    static const uint32_t sets[3][3] = {{17, 19, 23}, {29, 31, 37}, {41, 43, 47}};
    for (int i = 0; i < 3; ++i) {
      sv::PatPrimes pp;
      memset(&pp, 0, sizeof pp);
      for (int k = 0; k < 3; ++k) pp.p[k] = sets[i][k];
      pp.n = 3;
      const uint32_t end = i < 2 ? sv::kXOff[i + 1] : sv::kXWordsAll;
      const uint32_t nw = end - sv::kXOff[i];
      if (nw < (sv::kXPer[i] + sv::kPatWrapBits + 31) / 32) return SIEVE_E_HIP;   // layout constants
      STCHK(launch(c, "k_pattern", s, [&] {
        sv::k_pattern<<<(nw + 255) / 256, 256, 0, s>>>(c->xpat.as<uint32_t>() + sv::kXOff[i], sv::kXPer[i], pp, nw);
      }));
    }
    if (!g_dry) c->xpat_ready = true;
  }
  *xpat = c->xpat.as<uint32_t>();
  return SIEVE_OK;
}

// 17..47 come from patterns when every one of them sieves, the tile is 2^20 bits
// and the write-out takes four words per lane (segments of at least 2^13 bits, or
// tiles inside a segment).
bool use_xpat(uint64_t B, uint32_t L, uint32_t l) { return B >= 47 && L == 20 && (L < l || l >= 13); }

// Workgroups of 1024 lanes that one compute unit holds at tile size 2^L.
uint32_t tiles_per_cu(uint32_t L) {
  const size_t lds = ((size_t)1 << (L - 3)) + (sv::kPatWordsMax + sv::kSegSlotsMax + 1) * 4 +
                     (L == 20 ? sv::kXWordsAll : 4) * 4;
  return (uint32_t)std::max<size_t>(1, std::min<size_t>(2, (160 * 1024) / lds));
}

// Launches the tile kernel instantiated for tile size 2^L and entry type E over
// ta.ntiles tiles: one workgroup per resident slot, each taking a run of
// consecutive tiles.
template <typename E>
void launch_tile(const sieve_ctx* c, uint32_t L, hipStream_t s, sv::TileArgs ta) {
  const uint32_t g = std::max<uint32_t>(1, std::min<uint32_t>(ta.ntiles, c->ncu * tiles_per_cu(L)));
  switch (L) {
    case 13: sv::k_tile<E, 13><<<g, 1024, 0, s>>>(ta); break;
    case 14: sv::k_tile<E, 14><<<g, 1024, 0, s>>>(ta); break;
    case 15: sv::k_tile<E, 15><<<g, 1024, 0, s>>>(ta); break;
    case 16: sv::k_tile<E, 16><<<g, 1024, 0, s>>>(ta); break;
    case 17: sv::k_tile<E, 17><<<g, 1024, 0, s>>>(ta); break;
    case 18: sv::k_tile<E, 18><<<g, 1024, 0, s>>>(ta); break;
    case 19: sv::k_tile<E, 19><<<g, 1024, 0, s>>>(ta); break;
    default: sv::k_tile<E, 20><<<g, 1024, 0, s>>>(ta); break;
  }
}

// Device error word: allocated and cleared once per context.
int ensure_err(sieve_ctx* c, hipStream_t s) {
  if (c->err_ready) return SIEVE_OK;
  STCHK(c->err.ensure(64));
  if (g_dry) return SIEVE_OK;
  sv::k_fill_u32<<<1, 64, 0, s>>>(c->err.as<uint32_t>(), 16, 0);
  HIPCHK(hipGetLastError());
  c->err_ready = true;
  return SIEVE_OK;
}

// Builds the odd primes 3 <= p <= B into pr (device count in pr->cnt).
int build_primes(sieve_ctx* c, uint64_t B, sieve_primes* pr, hipStream_t s) {
  const uint64_t cap = pi_upper(B) + 16;
  STCHK(pr->P.ensure(cap * 4));
  STCHK(pr->cnt.ensure(16));
  uint32_t* P = pr->P.as<uint32_t>();
  uint32_t* cnt = pr->cnt.as<uint32_t>();
  if (B < 65536) {
    STCHK(launch(c, "k_base_primes", s, [&] {
      sv::k_base_primes<<<1, 1024, 0, s>>>((uint32_t)B, P, cnt, nullptr, nullptr, 0, 17, 0, 0, 0, 0);
    }));
  } else {
    // base primes up to isqrt(B) < 2^16, then one sieve of the odd numbers 1..B
    const uint64_t rb = isqrt_u64(B);
    STCHK(c->gen_blk.ensure(pi_upper(65536) * 4 + 64));
    uint32_t* base = c->gen_blk.as<uint32_t>();
    uint32_t* base_cnt = base + pi_upper(65536);
    // the generator table: bit k <-> 2k+1, k = 0..(B-1)/2, rounded up to whole
    // 2^15-bit count segments (the extra bits are masked off by the compaction);
    // tiles of 2^20 bits when there are a few hundred of them, else smaller tiles
    // so that a short table still spreads over many compute units
    const uint64_t kmax = (B - 1) / 2;
    constexpr uint32_t gl = 15;
    const uint64_t gbits = ((kmax + 1 + (1ull << gl) - 1) >> gl) << gl;
    uint32_t L = gl;
    while (L < kGenTile && (gbits >> (L + 9)) > 0) ++L;           // at least 256 tiles when possible
    const uint32_t nbase_ub = (uint32_t)pi_upper(65536);
    STCHK(c->plan.ensure(sizeof(sv::Plan) * 2));
    sv::Plan* gplan = c->plan.as<sv::Plan>() + 1;
    STCHK(c->Q0.ensure(pi_upper(65536) * 8));
    // base primes, the generator's plan and its launch offsets (from 0) in one kernel
    STCHK(launch(c, "k_base_primes", s, [&] {
      sv::k_base_primes<<<1, 1024, 0, s>>>((uint32_t)rb, base, base_cnt, gplan, c->Q0.as<uint2>(), nbase_ub,
                                           use_xpat(rb, L, gl) ? 53 : 17, 1u << 9, 1u << std::max(9u, L - 7),
                                           1u << 17, 1u << (L - 3));
    }));
    const uint32_t ntiles = (uint32_t)((gbits + (1ull << L) - 1) >> L);
    const uint32_t nwords = (uint32_t)(gbits / 32);
    const uint32_t nblk = (nwords + 1023) / 1024;
    const uint32_t ncnt = (uint32_t)(gbits >> gl);
    STCHK(c->gen_S.ensure(((size_t)nwords + nblk + ncnt + 64) * 4));
    uint32_t* gS = c->gen_S.as<uint32_t>();
    uint32_t* gcounts = gS + nwords + 32;
    const uint32_t* pat; uint32_t per, patw, pmask;
    STCHK(get_pattern(c, rb, s, &pat, &per, &patw, &pmask));
    sv::TileArgs ta;
    memset(&ta, 0, sizeof ta);
    ta.G0 = 0; ta.lbits = (uint32_t)gbits; ta.t0 = 0; ta.ntiles = ntiles; ta.L = L; ta.l = gl;
    ta.pat = pat; ta.per = per; ta.patw = patw; ta.per_G0 = 0; ta.per_tile = (uint32_t)((1ull << L) % per);
    ta.fixmask = pmask; ta.P = base; ta.QP = c->Q0.as<uint2>();
    ta.xon = use_xpat(rb, L, gl) ? 1u : 0u;
    if (ta.xon) STCHK(get_xpattern(c, s, &ta.xpat));
    ta.plan = gplan; ta.psq = 1; ta.has_large = 0; ta.b = 16;
    ta.S = gS; ta.counts = gcounts; ta.count_atomic = 0;
    ta.nwin = 1;
    ta.win[0] = {ta.G0, ta.lbits, ntiles, ta.psq, ta.per_G0, ta.S, ta.counts, ta.QP};
    STCHK(launch(c, "k_tile[gen]", s, [&] { launch_tile<uint16_t>(c, L, s, ta); }));
    // blocks of the compaction = count segments of the tile kernel (1024 words each)
    static_assert(gl == 15, "compaction blocks are 2^15-bit count segments");
    STCHK(ensure_err(c, s));
    STCHK(launch(c, "k_scan_small", s, [&] {
      sv::k_scan_small<<<1, 1024, 0, s>>>(gcounts, ncnt, cnt, (uint32_t)cap, gS, (uint32_t)kmax);
    }));
    STCHK(launch(c, "k_compact_write", s, [&] {
      sv::k_compact_write<<<nblk, 1024, 0, s>>>(gS, nwords, (uint32_t)kmax, gcounts, P, (uint32_t)cap,
                                                c->err.as<uint32_t>());
    }));
  }
  pr->B = B;
  return SIEVE_OK;
}

// Jobs of one chunk: ranges of at most sv::kMaxStageBins bins (at least
// `ranges`), each served by GR = groups / R workgroups with equal-work slices.
void chunk_jobs(uint32_t nbins, uint32_t cbits, uint32_t b, uint32_t ranges, uint32_t groups, double lo_p, double B,
                const uint32_t* Ptab, const sv::Plan* plan, const uint32_t* OFF_in, uint32_t* OFF_out,
                uint32_t gbin_base, std::vector<sv::BucketJob>* jobs, std::vector<uint32_t>* blk2job,
                std::vector<sv::BucketJob>* cjobs, std::vector<uint32_t>* cblk2job,
                std::vector<uint32_t>* thr, uint64_t* hg, uint32_t esz = 0) {
  // bin ranges: as given, or by default two for large chunks (a scatter workgroup
  // with fewer bins leaves fewer partly written lines in L2) and one otherwise; at
  // least enough for the LDS stages
  uint32_t R = ranges ? ranges : (nbins >= kAutoRangeBins ? 2u : 1u);
  R = std::max<uint32_t>(R, (nbins + sv::kMaxStageBins - 1) / sv::kMaxStageBins);
  R = std::min(R, nbins);
  const uint32_t rbins = (nbins + R - 1) / R;
  // workgroups per range (and of the count job): groups / ranges as given, or groups
  // by default; no more than one per kHitsPerGroup expected hits (small jobs would
  // otherwise pay a set-up and a flush per idle workgroup)
  const double range_hits = recip_sum_upper(lo_p, B) * (double)rbins * std::ldexp(1.0, (int)b);
  const uint32_t per_range = ranges ? std::max<uint32_t>(1, groups / R) : groups;
  const uint32_t GR = (uint32_t)std::max<double>(1.0, std::min<double>(per_range, std::ceil(range_hits / kHitsPerGroup)));
  const uint32_t t0 = (uint32_t)thr->size();
  thr->resize(t0 + GR);
  work_thresholds(lo_p, B, (double)rbins * (double)(1ull << b), GR, thr->data() + t0);
  // largest useful stage: about half a region's expected hits (larger stages would
  // not fill before the last flush); entries of 16 bits for bins up to 2^16 bits
  // unless 32-bit entries are asked for
  if (!esz) esz = b <= 16 ? 2 : 4;
  const double exp_region = recip_sum_upper(lo_p, B) * std::ldexp(1.0, (int)b) / GR;
  uint32_t sbl_cap = 0;
  while ((2u << sbl_cap) * esz <= sv::kMaxStageBytes && (double)(2u << sbl_cap) <= exp_region / 2) ++sbl_cap;
  // one count job over all bins (each prime visited once) whose histogram rows
  // (GR x nbins) the range jobs of the scatter read with row stride nbins
  const uint32_t hg0 = (uint32_t)*hg;
  {
    sv::BucketJob C;
    memset(&C, 0, sizeof C);
    C.Ptab = Ptab; C.plan = plan; C.OFF_in = OFF_in; C.OFF_out = OFF_out;
    C.thr = reinterpret_cast<const uint32_t*>((uintptr_t)t0);
    C.cbits = cbits; C.b = b; C.kb0 = 0; C.rbins = nbins; C.GR = GR;
    C.block0 = (uint32_t)cblk2job->size(); C.hg = hg0; C.hstride = nbins; C.gbin0 = gbin_base; C.sbl = 1;
    C.esz = esz;
    for (uint32_t q = 0; q < GR; ++q) cblk2job->push_back((uint32_t)cjobs->size());
    cjobs->push_back(C);
    *hg += (uint64_t)GR * nbins;
  }
  for (uint32_t x = 0; x < R; ++x) {
    sv::BucketJob J;
    memset(&J, 0, sizeof J);
    J.kb0 = x * rbins;
    if (J.kb0 >= nbins) break;
    J.Ptab = Ptab; J.plan = plan; J.OFF_in = OFF_in; J.OFF_out = OFF_out;
    J.thr = reinterpret_cast<const uint32_t*>((uintptr_t)t0);   // index into thr, rebased after upload
    J.cbits = cbits; J.b = b; J.rbins = std::min(rbins, nbins - J.kb0); J.update = (x + 1 == R) || (J.kb0 + rbins >= nbins);
    J.GR = GR; J.block0 = (uint32_t)blk2job->size(); J.hg = hg0 + J.kb0; J.hstride = nbins; J.gbin0 = gbin_base + J.kb0;
    J.sbl = sbl_cap;   // an upper bound here; set_stages fits it to the launch's LDS
    J.esz = esz;
    for (uint32_t q = 0; q < GR; ++q) blk2job->push_back((uint32_t)jobs->size());
    jobs->push_back(J);
    if (J.update) break;
  }
}

// Counting sort of the hits of a set of jobs into the bucket array:
// per-workgroup counts, scan over (bin, workgroup), staged scatter.
int bucket_fill_jobs(sieve_ctx* c, const sv::BucketJob* djobs, const uint32_t* dblk2job, uint32_t njobs, uint32_t nblocks,
                     const sv::BucketJob* dcjobs, const uint32_t* dcblk2job, uint32_t ncblocks, uint32_t max_cbins,
                     uint32_t gbins, uint32_t lds, uint32_t esz, uint32_t cap, hipStream_t s, bool logw = false) {
  uint32_t* HG = c->HG.as<uint32_t>();
  uint32_t* bst = c->bstart.as<uint32_t>();
  uint32_t* tot = bst + gbins + 1;
  const uint32_t gb = (gbins + sv::kBinsPerBlock - 1) / sv::kBinsPerBlock;
  const size_t lc = (size_t)max_cbins * 4, ls = lds;
  STCHK(launch(c, "k_bucket_count", s, [&] { sv::k_bucket_count2<<<ncblocks, 1024, lc, s>>>(dcjobs, dcblk2job, HG); }));
  STCHK(launch(c, "k_bin_total", s, [&] { sv::k_bin_jobs<<<gb, 1024, 0, s>>>(HG, djobs, njobs, gbins, tot, bst, 0); }));
  STCHK(launch(c, "k_bin_scan", s, [&] { sv::k_bin_scan<<<1, 1024, 0, s>>>(tot, gbins, bst); }));
  STCHK(launch(c, "k_bin_colprefix", s, [&] { sv::k_bin_jobs<<<gb, 1024, 0, s>>>(HG, djobs, njobs, gbins, tot, bst, 1); }));
  if (logw)
    STCHK(launch(c, "k_bucket_scatter", s, [&] {
      sv::k_bucket_scatter2<uint32_t, true><<<nblocks, 1024, ls, s>>>(djobs, dblk2job, HG, bst, c->bucket.as<uint32_t>(),
                                                                       cap, c->err.as<uint32_t>());
    }));
  else if (esz == 2)
    STCHK(launch(c, "k_bucket_scatter", s, [&] {
      sv::k_bucket_scatter2<uint16_t><<<nblocks, 1024, ls, s>>>(djobs, dblk2job, HG, bst, c->bucket.as<uint16_t>(),
                                                                 cap, c->err.as<uint32_t>());
    }));
  else
    STCHK(launch(c, "k_bucket_scatter", s, [&] {
      sv::k_bucket_scatter2<uint32_t><<<nblocks, 1024, ls, s>>>(djobs, dblk2job, HG, bst, c->bucket.as<uint32_t>(),
                                                                 cap, c->err.as<uint32_t>());
    }));
  return SIEVE_OK;
}

// Uploads jobs / block map / thresholds (rebasing the jobs' threshold pointers).
int upload_jobs(sieve_ctx* c, hipStream_t s) {
  STCHK(c->jobs.ensure(c->h_jobs.size() * sizeof(sv::BucketJob) + 64));
  STCHK(c->blk2job.ensure(c->h_blk2job.size() * 4 + 64));
  STCHK(c->cjobs.ensure(c->h_cjobs.size() * sizeof(sv::BucketJob) + 64));
  STCHK(c->cblk2job.ensure(c->h_cblk2job.size() * 4 + 64));
  STCHK(c->thr.ensure(c->h_thr.size() * 4 + 64));
  for (auto& J : c->h_jobs) J.thr = c->thr.as<uint32_t>() + reinterpret_cast<uintptr_t>(J.thr);
  for (auto& J : c->h_cjobs) J.thr = c->thr.as<uint32_t>() + reinterpret_cast<uintptr_t>(J.thr);
  STCHK(upload(c, s, c->jobs.p, c->h_jobs.data(), c->h_jobs.size() * sizeof(sv::BucketJob)));
  STCHK(upload(c, s, c->blk2job.p, c->h_blk2job.data(), c->h_blk2job.size() * 4));
  STCHK(upload(c, s, c->cjobs.p, c->h_cjobs.data(), c->h_cjobs.size() * sizeof(sv::BucketJob)));
  STCHK(upload(c, s, c->cblk2job.p, c->h_cblk2job.data(), c->h_cblk2job.size() * 4));
  STCHK(upload(c, s, c->thr.p, c->h_thr.data(), c->h_thr.size() * 4));
  return SIEVE_OK;
}

// Pinned staging bytes upload_jobs needs.
size_t job_upload_bytes(const sieve_ctx* c) {
  return pad256(c->h_jobs.size() * sizeof(sv::BucketJob)) + pad256(c->h_blk2job.size() * 4) +
         pad256(c->h_cjobs.size() * sizeof(sv::BucketJob)) + pad256(c->h_cblk2job.size() * 4) +
         pad256(c->h_thr.size() * 4);
}

// Bin size of the sparse primes' sort for a window of lbits bits: about 256 bins, of
// 2^15 .. 2^20 bits (the apply step holds one bin in LDS).
uint32_t sp_binlog(uint64_t lbits) {
  uint32_t lg = 0;
  while ((1ull << lg) < lbits) ++lg;
  return std::min<uint32_t>(20, std::max<uint32_t>(15, lg > 8 ? lg - 8 : 0));
}

// The sieve proper for one request (l, F, NB) with the table pr and bound B.
// wide (two words, lo then hi), when given, is the true 128-bit start F of an
// interval beyond 2^64: the first offsets come from it, every p^2 start rule is off
// (psq = 2^32 - 1) and F is a stand-in congruent to it modulo 3*5*...*47, which is
// all the tile kernel reads of the start besides those rules.
int run_sieve(sieve_ctx* c, const sieve_primes* pr, uint32_t l, uint64_t F, uint64_t NB, uint64_t B,
              uint32_t* S, uint32_t* counts, const Resolved& R, hipStream_t s, const uint64_t* wide = nullptr) {
  const uint32_t L = R.L;
  const uint64_t wave_lim = 1ull << R.Wlog, wheel_lim = 1ull << R.Blog, med_lim = 1ull << R.Mlog;
  const uint64_t tab_ub = std::min<uint64_t>(pi_upper(B), pi_upper(pr->B));
  // sparse large primes: p at least the launch window length (at most one hit per
  // window), taken by k_sparse_collect / k_sparse_apply after the tile kernel instead
  // of the buckets unless the tuning turns that off (the bucket path computes the same
  // first offsets and then walks every prime twice more)
  const uint64_t sparse_lim = std::max<uint64_t>(med_lim, std::min<uint64_t>(NB, kLaunchBits));
  const bool sparse = !wide && R.sparse != 1 && sparse_lim > med_lim && B >= sparse_lim;
  STCHK(c->plan.ensure(sizeof(sv::Plan) * 2));
  sv::Plan* plan = c->plan.as<sv::Plan>();
  STCHK(launch(c, "k_plan", s, [&] {
    sv::k_plan<<<1, 64, 0, s>>>(pr->P.as<uint32_t>(), pr->cnt.as<uint32_t>(), B, use_xpat(B, L, l) ? 53 : 17, wave_lim,
                               wheel_lim, med_lim, 1ull << (L - 3), (uint32_t)tab_ub, plan, sparse ? sparse_lim : ~0ull);
  }));
  const uint64_t B_dense = sparse ? sparse_lim - 1 : B;          // the bucket fill's primes end there
  const uint64_t med_ub = std::min<uint64_t>(tab_ub, pi_upper(med_lim));
  STCHK(c->Q0.ensure(med_ub * 8 + 64));
  const bool large = B >= med_lim;
  // bucketed primes: indices iM .. iS, and iS <= pi(sparse_lim - 1) when sparse
  const uint64_t nL_ub = large ? (sparse ? std::min<uint64_t>(tab_ub, pi_upper(sparse_lim)) : tab_ub) : 0;
  if (large) STCHK(c->OFF.ensure(2 * nL_ub * 4 + 64));           // in / out halves
  const uint32_t* pat; uint32_t per, patw, pmask;
  STCHK(get_pattern(c, B, s, &pat, &per, &patw, &pmask));
  const uint32_t nwin = (uint32_t)((NB + kLaunchBits - 1) / kLaunchBits);
  if (!large && nwin <= sv::kMaxWins) {
    // medium primes only: one offsets launch and one tile launch for all windows
    STCHK(c->Q0.ensure((size_t)nwin * med_ub * 8 + 64));
    STCHK(ensure_err(c, s));
    const bool count_atomic = L < l;
    if (count_atomic) {
      const uint64_t n = NB >> l;
      STCHK(launch(c, "k_fill_u32", s, [&] { sv::k_fill_u32<<<(uint32_t)std::min<uint64_t>((n + 255) / 256, 4096), 256, 0, s>>>(counts, n, 0); }));
    }
    const dim3 og((uint32_t)((tab_ub + 256 * sv::kOffPer - 1) / (256 * sv::kOffPer)), nwin);
    if (wide)
      STCHK(launch(c, "k_offsets_wide", s, [&] {
        sv::k_offsets_wide<<<og, 256, 0, s>>>(pr->P.as<uint32_t>(), plan, wide[0], wide[1], kLaunchBits,
                                              c->Q0.as<uint2>(), nullptr, (uint32_t)med_ub);
      }));
    else
      STCHK(launch(c, "k_offsets", s, [&] {
        sv::k_offsets<<<og, 256, 0, s>>>(pr->P.as<uint32_t>(), plan, F, kLaunchBits, c->Q0.as<uint2>(), nullptr,
                                         (uint32_t)med_ub);
      }));
    sv::TileArgs ta;
    memset(&ta, 0, sizeof ta);
    ta.G0 = F; ta.t0 = 0; ta.L = L; ta.l = l;
    ta.pat = pat; ta.per = per; ta.patw = patw; ta.per_tile = (uint32_t)((1ull << L) % per);
    ta.fixmask = pmask; ta.P = pr->P.as<uint32_t>(); ta.QP = c->Q0.as<uint2>();
    ta.xon = use_xpat(B, L, l) ? 1u : 0u;
    if (ta.xon) STCHK(get_xpattern(c, s, &ta.xpat));
    ta.plan = plan; ta.b = R.b; ta.has_large = 0; ta.count_atomic = count_atomic ? 1 : 0;
    ta.nwin = nwin;
    uint32_t ntot = 0;
    for (uint32_t w = 0; w < nwin; ++w) {
      const uint64_t ls = (uint64_t)w * kLaunchBits, lb = std::min<uint64_t>(kLaunchBits, NB - ls);
      sv::TileWin& W = ta.win[w];
      W.G0 = F + ls;
      W.lbits = (uint32_t)lb;
      W.ntiles = (uint32_t)((lb + (1ull << L) - 1) >> L);
      W.psq = wide ? 0xFFFFFFFFu : (uint32_t)std::min<uint64_t>(isqrt_u64(2 * W.G0 + 1), 0xFFFFFFFFull);
      W.per_G0 = (uint32_t)(W.G0 % per);
      W.S = S + (ls >> 5);
      W.counts = counts + (ls >> l);
      W.QP = c->Q0.as<uint2>() + (size_t)w * med_ub;
      ntot += W.ntiles;
    }
    ta.ntiles = ntot;
    ta.lbits = ta.win[0].lbits; ta.psq = ta.win[0].psq; ta.per_G0 = ta.win[0].per_G0;
    ta.S = S; ta.counts = counts;
    STCHK(launch(c, "k_tile", s, [&] { launch_tile<uint32_t>(c, L, s, ta); }));
    return SIEVE_OK;
  }
  const uint32_t b = R.b;
  const uint32_t esz = b <= 16 ? 2 : 4;                        // bytes per bucket entry
  const uint64_t chunk_max = std::min<uint64_t>((1ull << R.binslog) << b, kLaunchBits);  // bits per bucket fill
  // every chunk of every launch, with its bucket jobs
  struct Chunk { uint64_t ls, lbits, cs, cbits; uint32_t nbins, j0, j1, b0, b1, cj0, cb0, cb1, max_rbins, lds; };
  std::vector<Chunk> chunks;
  c->h_jobs.clear(); c->h_blk2job.clear(); c->h_cjobs.clear(); c->h_cblk2job.clear(); c->h_thr.clear();
  uint64_t hg_max = 0, cap = 0, pad_max = 0;
  uint32_t nbins_max = 0;
  if (large) {
    const double rs = recip_sum_upper((double)med_lim, (double)B_dense);
    cap = (uint64_t)(1.02 * rs * (double)std::min<uint64_t>(chunk_max, NB)) + nL_ub + 4096;
    if (cap >= 0xFFFFFFFFull) return SIEVE_E_NOMEM;
  }
  for (uint64_t ls = 0; ls < NB; ls += kLaunchBits) {
    const uint64_t lbits = std::min<uint64_t>(kLaunchBits, NB - ls);
    uint32_t off_cur = 0;   // which half of OFF holds the offsets of the current chunk
    for (uint64_t cs = 0; cs < lbits; cs += chunk_max) {
      Chunk ch;
      ch.ls = ls; ch.lbits = lbits; ch.cs = cs; ch.cbits = std::min<uint64_t>(chunk_max, lbits - cs);
      ch.nbins = (uint32_t)((ch.cbits + (1ull << b) - 1) >> b);
      ch.j0 = (uint32_t)c->h_jobs.size(); ch.b0 = (uint32_t)c->h_blk2job.size();
      ch.cj0 = (uint32_t)c->h_cjobs.size(); ch.cb0 = (uint32_t)c->h_cblk2job.size();
      ch.max_rbins = 1;
      if (large) {
        uint64_t hg = 0;
        const uint32_t* oin = c->OFF.as<uint32_t>() + (size_t)off_cur * nL_ub;
        uint32_t* oout = c->OFF.as<uint32_t>() + (size_t)(1 - off_cur) * nL_ub;
        const size_t jb = c->h_jobs.size(), cjb = c->h_cjobs.size();
        chunk_jobs(ch.nbins, (uint32_t)ch.cbits, b, R.R, R.groups, (double)med_lim, (double)B_dense,
                   pr->P.as<uint32_t>(), plan, oin, oout, 0, &c->h_jobs, &c->h_blk2job, &c->h_cjobs, &c->h_cblk2job,
                   &c->h_thr, &hg);
        for (size_t k = jb; k < c->h_jobs.size(); ++k) {   // block numbers and job indices relative to the chunk
          c->h_jobs[k].block0 -= ch.b0;
          ch.max_rbins = std::max(ch.max_rbins, c->h_jobs[k].rbins);
        }
        for (size_t k = cjb; k < c->h_cjobs.size(); ++k) c->h_cjobs[k].block0 -= ch.cb0;
        pad_max = std::max(pad_max, set_stages(c->h_jobs, jb, c->h_jobs.size(), esz, &ch.lds));
        for (size_t k = ch.b0; k < c->h_blk2job.size(); ++k) c->h_blk2job[k] -= ch.j0;
        for (size_t k = ch.cb0; k < c->h_cblk2job.size(); ++k) c->h_cblk2job[k] -= ch.cj0;
        hg_max = std::max(hg_max, hg);
        nbins_max = std::max(nbins_max, ch.nbins);
        off_cur ^= 1u;
      }
      ch.j1 = (uint32_t)c->h_jobs.size(); ch.b1 = (uint32_t)c->h_blk2job.size();
      ch.cb1 = (uint32_t)c->h_cblk2job.size();
      chunks.push_back(ch);
    }
  }
  if (large) {
    cap += pad_max;
    if (cap >= 0xFFFFFFFFull) return SIEVE_E_NOMEM;
    STCHK(c->HG.ensure(hg_max * 4 + 64));
    STCHK(c->bstart.ensure(((size_t)2 * nbins_max + 2) * 4));   // bin_start, then bin totals
    STCHK(c->bucket.ensure(cap * esz));
    STCHK(pin_begin(c, job_upload_bytes(c)));
    STCHK(upload_jobs(c, s));
    STCHK(pin_end(c, s));
  }
  // sparse primes: at most tab_ub - (pi(sparse_lim - 1) - 1) of them, with
  // pi(x) > x / ln x for x >= 17 (Rosser and Schoenfeld)
  uint32_t sp_nwg = 0;
  if (sparse) {
    const double x = (double)(sparse_lim - 1);
    const uint64_t below = (uint64_t)(x / std::log(x));
    const uint64_t nsp_ub = tab_ub > below ? tab_ub - below + 2 : 2;
    const uint64_t nwg = (nsp_ub + 8 * sv::kSpK - 1) / (8 * sv::kSpK) * 8;   // a multiple of the XCD count
    if (nwg * sv::kSpK >= 0xFFFFFFFFull) return SIEVE_E_NOMEM;
    sp_nwg = (uint32_t)nwg;
    uint64_t hdr_words = 0;
    for (uint64_t ls = 0; ls < NB; ls += kLaunchBits) {
      const uint64_t lb = std::min<uint64_t>(kLaunchBits, NB - ls);
      hdr_words = std::max<uint64_t>(hdr_words, ((lb + (1ull << sp_binlog(lb)) - 1) >> sp_binlog(lb)) * nwg);
    }
    STCHK(c->spE.ensure(nwg * sv::kSpK * 4));
    STCHK(c->spH.ensure(hdr_words * 4 + 64));
  }
  STCHK(ensure_err(c, s));
  const bool count_atomic = L < l;
  if (count_atomic) {
    const uint64_t n = NB >> l;
    STCHK(launch(c, "k_fill_u32", s, [&] { sv::k_fill_u32<<<(uint32_t)std::min<uint64_t>((n + 255) / 256, 4096), 256, 0, s>>>(counts, n, 0); }));
  }
  const uint32_t patG_step = (uint32_t)((1ull << L) % per);
  const sv::BucketJob* djobs = c->jobs.as<sv::BucketJob>();
  const uint32_t* dblk = c->blk2job.as<uint32_t>();
  const sv::BucketJob* dcjobs = c->cjobs.as<sv::BucketJob>();
  const uint32_t* dcblk = c->cblk2job.as<uint32_t>();
  uint64_t cur_ls = ~0ull;
  for (const Chunk& ch : chunks) {
    const uint64_t G0 = F + ch.ls;
    if (ch.ls != cur_ls) {
      cur_ls = ch.ls;
      // grid over the primes >= 17 that k_offsets works: below the sparse ones
      const uint64_t off_ub = sparse ? std::min<uint64_t>(tab_ub, pi_upper(sparse_lim)) : tab_ub;
      const uint32_t og = (uint32_t)((off_ub + 256 * sv::kOffPer - 1) / (256 * sv::kOffPer));
      uint32_t* off = large ? c->OFF.as<uint32_t>() : nullptr;
      if (wide) {
        const uint64_t lo = wide[0] + ch.ls, hi = wide[1] + (lo < wide[0] ? 1u : 0u);
        STCHK(launch(c, "k_offsets_wide", s, [&] {
          sv::k_offsets_wide<<<og, 256, 0, s>>>(pr->P.as<uint32_t>(), plan, lo, hi, ch.lbits, c->Q0.as<uint2>(), off, 0);
        }));
      } else {
        STCHK(launch(c, "k_offsets", s, [&] {
          sv::k_offsets<<<og, 256, 0, s>>>(pr->P.as<uint32_t>(), plan, G0, ch.lbits, c->Q0.as<uint2>(), off, 0);
        }));
      }
    }
    const uint64_t psq = wide ? 0xFFFFFFFFull : isqrt_u64(2 * G0 + 1);
    const uint32_t ntiles = (uint32_t)((ch.cbits + (1ull << L) - 1) >> L);
    if (large)
      STCHK(bucket_fill_jobs(c, djobs + ch.j0, dblk + ch.b0, ch.j1 - ch.j0, ch.b1 - ch.b0, dcjobs + ch.cj0, dcblk + ch.cb0,
                             ch.cb1 - ch.cb0, ch.nbins, ch.nbins, ch.lds, esz, (uint32_t)cap, s));
    sv::TileArgs ta;
    memset(&ta, 0, sizeof ta);
    ta.G0 = G0; ta.lbits = (uint32_t)ch.lbits; ta.t0 = (uint32_t)(ch.cs >> L); ta.ntiles = ntiles; ta.L = L; ta.l = l;
    ta.pat = pat; ta.per = per; ta.patw = patw; ta.per_G0 = (uint32_t)(G0 % per); ta.per_tile = patG_step;
    ta.fixmask = pmask; ta.P = pr->P.as<uint32_t>(); ta.QP = c->Q0.as<uint2>();
    ta.xon = use_xpat(B, L, l) ? 1u : 0u;
    if (ta.xon) STCHK(get_xpattern(c, s, &ta.xpat));
    ta.plan = plan; ta.psq = (uint32_t)std::min<uint64_t>(psq, 0xFFFFFFFFull);
    ta.bucket = large ? c->bucket.p : nullptr; ta.bin_start = large ? c->bstart.as<uint32_t>() : nullptr;
    ta.b = b; ta.nbins = ch.nbins; ta.cap = (uint32_t)cap; ta.has_large = large ? 1 : 0;
    ta.S = S + (ch.ls >> 5); ta.counts = counts + (ch.ls >> l); ta.count_atomic = count_atomic ? 1 : 0;
    ta.nwin = 1;
    ta.win[0] = {ta.G0, ta.lbits, ntiles, ta.psq, ta.per_G0, ta.S, ta.counts, ta.QP};
    if (esz == 2)
      STCHK(launch(c, "k_tile", s, [&] { launch_tile<uint16_t>(c, L, s, ta); }));
    else
      STCHK(launch(c, "k_tile", s, [&] { launch_tile<uint32_t>(c, L, s, ta); }));
    if (sparse && (&ch == &chunks.back() || (&ch + 1)->ls != ch.ls)) {
      // the window is written: the sparse primes' hits, sorted by bin, OR-ed in; then
      // its counts again
      uint32_t* Sw = S + (ch.ls >> 5);
      const uint32_t binlog = sp_binlog(ch.lbits);
      const uint32_t nbins = (uint32_t)((ch.lbits + (1ull << binlog) - 1) >> binlog);
      // the p^2 start rule can move a sparse prime's hit only if p^2 > u, i.e. p >
      // isqrt(2 G0 + 1) for some prime p >= sparse_lim of the table (p <= B)
      const bool sq = isqrt_u64(2 * G0 + 1) < B;
      STCHK(launch(c, "k_sparse_collect", s, [&] {
        if (sq)
          sv::k_sparse_collect<true><<<sp_nwg, sv::kSpThreads, 0, s>>>(
              pr->P.as<uint32_t>(), plan, G0, ch.lbits, binlog, nbins, sp_nwg, c->spE.as<uint32_t>(),
              c->spH.as<uint32_t>(), c->err.as<uint32_t>());
        else
          sv::k_sparse_collect<false><<<sp_nwg, sv::kSpThreads, 0, s>>>(
              pr->P.as<uint32_t>(), plan, G0, ch.lbits, binlog, nbins, sp_nwg, c->spE.as<uint32_t>(),
              c->spH.as<uint32_t>(), c->err.as<uint32_t>());
      }));
      STCHK(launch(c, "k_sparse_apply", s, [&] {
        sv::k_sparse_apply<<<nbins, sv::kSpApplyThreads, (1u << binlog) / 8, s>>>(
            c->spE.as<uint32_t>(), c->spH.as<uint32_t>(), sp_nwg, binlog, ch.lbits, Sw);
      }));
      const uint32_t nseg = (uint32_t)(ch.lbits >> l);
      STCHK(launch(c, "k_recount", s, [&] {
        sv::k_recount<<<l >= 13 ? nseg : (nseg + 255) / 256, 256, 0, s>>>(Sw, l, nseg, counts + (ch.ls >> l));
      }));
    }
  }
  return SIEVE_OK;
}

// The log-add sieve of (l, F, NB) with the odd primes <= B of pr (Section 5's wider
// use of buckets): tiles of 2^L positions whose byte sums sit in LDS, the medium
// primes (below 2^L) walked per tile from their first offsets in the window, the
// larger ones counting-sorted into per-tile bins of 32-bit entries carrying their
// weight, chunks of 2^11 bins; output the candidate table C (sum >= T), the ones per
// segment and optionally the sums A.
constexpr uint32_t kLogBinsLog = 11;
int run_logsieve(sieve_ctx* c, const sieve_primes* pr, uint32_t l, uint64_t F, uint64_t NB, uint64_t B, uint32_t T,
                 uint32_t* C, uint32_t* counts, uint8_t* A, uint32_t L, uint32_t groups, uint32_t ranges, hipStream_t s) {
  const uint64_t med_lim = 1ull << L;
  const uint64_t tab_ub = std::min<uint64_t>(pi_upper(B), pi_upper(pr->B));
  STCHK(c->plan.ensure(sizeof(sv::Plan) * 2));
  sv::Plan* plan = c->plan.as<sv::Plan>();
  STCHK(launch(c, "k_plan", s, [&] {
    sv::k_plan<<<1, 64, 0, s>>>(pr->P.as<uint32_t>(), pr->cnt.as<uint32_t>(), B, 17, 1ull << 9, 1ull << 9, med_lim,
                               1ull << (L - 3), (uint32_t)tab_ub, plan);
  }));
  // the weights of the primes 3..13 up to B, one period, with which every tile starts
  const uint32_t nsmall = (B >= 3) + (B >= 5) + (B >= 7) + (B >= 11) + (B >= 13);
  STCHK(c->logpat.ensure(sv::kLogPatWords * 4));
  STCHK(launch(c, "k_logpattern", s, [&] {
    sv::k_logpattern<<<(sv::kLogPatWords + 255) / 256, 256, 0, s>>>(c->logpat.as<uint32_t>(), nsmall);
  }));
  const uint64_t med_ub = std::min<uint64_t>(tab_ub, pi_upper(med_lim));
  STCHK(c->Q0.ensure(med_ub * 8 + 64));
  const bool large = B >= med_lim;
  const uint64_t nL_ub = large ? tab_ub : 0;
  if (large) STCHK(c->OFF.ensure(2 * nL_ub * 4 + 64));
  const uint32_t b = L, esz = 4;
  const uint64_t chunk_max = std::min<uint64_t>(1ull << (kLogBinsLog + b), kLaunchBits);
  struct Chunk { uint64_t ls, lbits, cs, cbits; uint32_t nbins, j0, j1, b0, b1, cj0, cb0, cb1, lds; };
  std::vector<Chunk> chunks;
  c->h_jobs.clear(); c->h_blk2job.clear(); c->h_cjobs.clear(); c->h_cblk2job.clear(); c->h_thr.clear();
  uint64_t hg_max = 0, cap = 0, pad_max = 0;
  uint32_t nbins_max = 0;
  if (large) {
    cap = (uint64_t)(1.02 * recip_sum_upper((double)med_lim, (double)B) * (double)std::min<uint64_t>(chunk_max, NB)) +
          nL_ub + 4096;
    if (cap >= 0xFFFFFFFFull) return SIEVE_E_NOMEM;
  }
  for (uint64_t ls = 0; ls < NB; ls += kLaunchBits) {
    const uint64_t lbits = std::min<uint64_t>(kLaunchBits, NB - ls);
    uint32_t off_cur = 0;
    for (uint64_t cs = 0; cs < lbits; cs += chunk_max) {
      Chunk ch;
      ch.ls = ls; ch.lbits = lbits; ch.cs = cs; ch.cbits = std::min<uint64_t>(chunk_max, lbits - cs);
      ch.nbins = (uint32_t)((ch.cbits + (1ull << b) - 1) >> b);
      ch.j0 = (uint32_t)c->h_jobs.size(); ch.b0 = (uint32_t)c->h_blk2job.size();
      ch.cj0 = (uint32_t)c->h_cjobs.size(); ch.cb0 = (uint32_t)c->h_cblk2job.size();
      ch.lds = 0;
      if (large) {
        uint64_t hg = 0;
        const uint32_t* oin = c->OFF.as<uint32_t>() + (size_t)off_cur * nL_ub;
        uint32_t* oout = c->OFF.as<uint32_t>() + (size_t)(1 - off_cur) * nL_ub;
        const size_t jb = c->h_jobs.size(), cjb = c->h_cjobs.size();
        chunk_jobs(ch.nbins, (uint32_t)ch.cbits, b, ranges, groups, (double)med_lim, (double)B, pr->P.as<uint32_t>(),
                   plan, oin, oout, 0, &c->h_jobs, &c->h_blk2job, &c->h_cjobs, &c->h_cblk2job, &c->h_thr, &hg, esz);
        for (size_t k = jb; k < c->h_jobs.size(); ++k) c->h_jobs[k].block0 -= ch.b0;
        for (size_t k = cjb; k < c->h_cjobs.size(); ++k) c->h_cjobs[k].block0 -= ch.cb0;
        pad_max = std::max(pad_max, set_stages(c->h_jobs, jb, c->h_jobs.size(), esz, &ch.lds));
        for (size_t k = ch.b0; k < c->h_blk2job.size(); ++k) c->h_blk2job[k] -= ch.j0;
        for (size_t k = ch.cb0; k < c->h_cblk2job.size(); ++k) c->h_cblk2job[k] -= ch.cj0;
        hg_max = std::max(hg_max, hg);
        nbins_max = std::max(nbins_max, ch.nbins);
        off_cur ^= 1u;
      }
      ch.j1 = (uint32_t)c->h_jobs.size(); ch.b1 = (uint32_t)c->h_blk2job.size();
      ch.cb1 = (uint32_t)c->h_cblk2job.size();
      chunks.push_back(ch);
    }
  }
  if (large) {
    cap += pad_max;
    if (cap >= 0xFFFFFFFFull) return SIEVE_E_NOMEM;
    STCHK(c->HG.ensure(hg_max * 4 + 64));
    STCHK(c->bstart.ensure(((size_t)2 * nbins_max + 2) * 4));
    STCHK(c->bucket.ensure(cap * esz));
    STCHK(pin_begin(c, job_upload_bytes(c)));
    STCHK(upload_jobs(c, s));
    STCHK(pin_end(c, s));
  }
  STCHK(ensure_err(c, s));
  if (l > L) {
    const uint64_t n = NB >> l;
    STCHK(launch(c, "k_fill_u32", s, [&] {
      sv::k_fill_u32<<<(uint32_t)std::min<uint64_t>((n + 255) / 256, 4096), 256, 0, s>>>(counts, n, 0);
    }));
  }
  const sv::BucketJob* djobs = c->jobs.as<sv::BucketJob>();
  const uint32_t* dblk = c->blk2job.as<uint32_t>();
  const sv::BucketJob* dcjobs = c->cjobs.as<sv::BucketJob>();
  const uint32_t* dcblk = c->cblk2job.as<uint32_t>();
  uint64_t cur_ls = ~0ull;
  for (const Chunk& ch : chunks) {
    const uint64_t G0 = F + ch.ls;
    if (ch.ls != cur_ls) {
      cur_ls = ch.ls;
      STCHK(launch(c, "k_offsets", s, [&] {
        sv::k_offsets<<<(uint32_t)((tab_ub + 256 * sv::kOffPer - 1) / (256 * sv::kOffPer)), 256, 0, s>>>(
            pr->P.as<uint32_t>(), plan, G0, ch.lbits, c->Q0.as<uint2>(), large ? c->OFF.as<uint32_t>() : nullptr, 0, 1);
      }));
    }
    if (large)
      STCHK(bucket_fill_jobs(c, djobs + ch.j0, dblk + ch.b0, ch.j1 - ch.j0, ch.b1 - ch.b0, dcjobs + ch.cj0, dcblk + ch.cb0,
                             ch.cb1 - ch.cb0, ch.nbins, ch.nbins, ch.lds, esz, (uint32_t)cap, s, true));
    sv::LogArgs a;
    memset(&a, 0, sizeof a);
    a.G0 = G0; a.lbits = (uint32_t)ch.lbits; a.t0 = (uint32_t)(ch.cs >> L); a.l = l; a.T = T;
    a.QP = c->Q0.as<uint2>(); a.plan = plan;
    a.bucket = large ? c->bucket.p : nullptr; a.bin_start = large ? c->bstart.as<uint32_t>() : nullptr;
    a.nbins = ch.nbins; a.cap = (uint32_t)cap; a.has_large = large ? 1 : 0; a.count_atomic = l > L ? 1 : 0;
    a.C = C + (ch.ls >> 5); a.counts = counts + (ch.ls >> l); a.A = A ? A + ch.ls : nullptr;
    a.pat = c->logpat.as<uint32_t>();
    const uint32_t ntiles = (uint32_t)((ch.cbits + (1ull << L) - 1) >> L);
    STCHK(launch(c, "k_logtile", s, [&] {
      switch (L) {
        case 14: sv::k_logtile<14><<<ntiles, 1024, 0, s>>>(a); break;
        case 15: sv::k_logtile<15><<<ntiles, 1024, 0, s>>>(a); break;
        case 16: sv::k_logtile<16><<<ntiles, 1024, 0, s>>>(a); break;
        default: sv::k_logtile<17><<<ntiles, 1024, 0, s>>>(a); break;
      }
    }));
  }
  return SIEVE_OK;
}

int begin(sieve_ctx* c, hipStream_t s) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  c->device = dev;
  if (!c->ncu) {
    int ncu = 0;
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    c->ncu = (uint32_t)std::max(ncu, 1);
  }
  if (g_dry) return SIEVE_OK;
  STCHK(set_lds_limits());
  if (c->has_last && c->last_stream != s) HIPCHK(hipStreamWaitEvent(s, c->done, 0));
  g_call_stream = s;
  g_in_call = true;
  return SIEVE_OK;
}

int end(sieve_ctx* c, hipStream_t s) {
  g_in_call = false;
  if (g_dry) return SIEVE_OK;
  if (!c->done) HIPCHK(hipEventCreateWithFlags(&c->done, hipEventDisableTiming));
  HIPCHK(hipEventRecord(c->done, s));
  c->last_stream = s;
  c->has_last = true;
  return SIEVE_OK;
}

// Runs fn on a fresh context in dry-run mode: the device bytes its buffers would
// hold afterwards (nothing is allocated or enqueued).
template <typename F>
int dry_bytes(F&& fn, uint64_t* bytes) {
  sieve_ctx tmp;
  DryRun d;
  g_dry = &d;
  const int rc = fn(&tmp);
  g_dry = nullptr;
  if (rc != SIEVE_OK) return rc;
  uint64_t tot = 0;
  for (auto& w : d.want) tot += w.second;
  *bytes = tot;
  return SIEVE_OK;
}

std::mutex g_default_mu;
std::map<int, sieve_ctx*> g_default;

}  // namespace

extern "C" {

int sieve_ctx_create(sieve_ctx** out) {
  if (!out) return SIEVE_E_ARG;
  *out = new (std::nothrow) sieve_ctx();
  return *out ? SIEVE_OK : SIEVE_E_NOMEM;
}

int sieve_ctx_destroy(sieve_ctx* ctx) {
  if (!ctx) return SIEVE_E_ARG;
  delete ctx;
  return SIEVE_OK;
}

sieve_ctx* sieve_default_ctx(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> g(g_default_mu);
  auto it = g_default.find(dev);
  if (it != g_default.end()) return it->second;
  sieve_ctx* c = new (std::nothrow) sieve_ctx();
  if (c) g_default[dev] = c;
  return c;
}

int sieve_ctx_sieve(sieve_ctx* ctx, uint32_t l, uint64_t f, uint64_t n, uint64_t B, uint32_t* S_dev,
                    uint32_t* counts_dev, const sieve_tune* tune, void* stream) {
  if (!ctx || !S_dev || !counts_dev) return SIEVE_E_ARG;
  uint64_t F, NB;
  STCHK(check_interval(l, f, n, B, &F, &NB));
  Resolved R;
  STCHK(resolve_tune(l, tune, &R));
  std::lock_guard<std::mutex> g(ctx->mu);
  hipStream_t s = (hipStream_t)stream;
  STCHK(begin(ctx, s));
  STCHK(build_primes(ctx, B, &ctx->own, s));
  STCHK(run_sieve(ctx, &ctx->own, l, F, NB, B, S_dev, counts_dev, R, s));
  return end(ctx, s);
}

int sieve_init(uint32_t l, uint64_t f, uint64_t n, uint64_t B, uint32_t* S_dev, uint32_t* counts_dev,
               void* stream) {
  // argument checks come before any HIP call
  if (!S_dev || !counts_dev) return SIEVE_E_ARG;
  uint64_t F, NB;
  STCHK(check_interval(l, f, n, B, &F, &NB));
  sieve_ctx* c = sieve_default_ctx();
  if (!c) return SIEVE_E_HIP;
  return sieve_ctx_sieve(c, l, f, n, B, S_dev, counts_dev, nullptr, stream);
}

int sieve_primes_create(uint64_t B, void* stream, sieve_primes** out) {
  if (!out) return SIEVE_E_ARG;
  *out = nullptr;
  if (B < 3 || B >= (1ull << 32)) return SIEVE_E_BOUND;
  sieve_ctx* c = sieve_default_ctx();
  if (!c) return SIEVE_E_HIP;
  sieve_primes* pr = new (std::nothrow) sieve_primes();
  if (!pr) return SIEVE_E_NOMEM;
  hipStream_t s = (hipStream_t)stream;
  int rc;
  {
    std::lock_guard<std::mutex> g(c->mu);
    rc = begin(c, s);
    if (rc == SIEVE_OK) rc = build_primes(c, B, pr, s);
    if (rc == SIEVE_OK) rc = end(c, s);
  }
  uint32_t cnt = 0;
  if (rc == SIEVE_OK) {
    hipError_t e = hipMemcpyAsync(&cnt, pr->cnt.p, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { g_last_hip = (int)e; rc = SIEVE_E_HIP; }
  }
  if (rc != SIEVE_OK) { pr->P.release(); pr->cnt.release(); delete pr; return rc; }
  pr->count = cnt;
  pr->device = c->device;
  *out = pr;
  return SIEVE_OK;
}

int sieve_primes_destroy(sieve_primes* pr) {
  if (!pr) return SIEVE_E_ARG;
  (void)hipDeviceSynchronize();
  pr->P.release(); pr->cnt.release();
  delete pr;
  return SIEVE_OK;
}

int sieve_primes_info(const sieve_primes* pr, uint64_t* count, uint64_t* bound) {
  if (!pr) return SIEVE_E_ARG;
  if (count) *count = pr->count;
  if (bound) *bound = pr->B;
  return SIEVE_OK;
}

int sieve_primes_copy(const sieve_primes* pr, uint32_t* dst_dev, uint64_t cap, void* stream) {
  if (!pr || !dst_dev) return SIEVE_E_ARG;
  uint64_t n = std::min(cap, pr->count);
  if (n) HIPCHK(hipMemcpyAsync(dst_dev, pr->P.p, n * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return SIEVE_OK;
}

int sieve_ctx_sieve_with(sieve_ctx* ctx, const sieve_primes* pr, uint32_t l, uint64_t f, uint64_t n, uint64_t B,
                         uint32_t* S_dev, uint32_t* counts_dev, const sieve_tune* tune, void* stream) {
  if (!ctx || !pr || !S_dev || !counts_dev) return SIEVE_E_ARG;
  uint64_t F, NB;
  STCHK(check_interval(l, f, n, B, &F, &NB));
  if (B > pr->B) return SIEVE_E_BOUND;
  Resolved R;
  STCHK(resolve_tune(l, tune, &R));
  std::lock_guard<std::mutex> g(ctx->mu);
  hipStream_t s = (hipStream_t)stream;
  STCHK(begin(ctx, s));
  STCHK(run_sieve(ctx, pr, l, F, NB, B, S_dev, counts_dev, R, s));
  return end(ctx, s);
}

int sieve_required_bound(uint32_t l, uint64_t f, uint64_t n, uint64_t* B) {
  if (!B) return SIEVE_E_ARG;
  if (l < 5 || l > 20 || n == 0) return SIEVE_E_ARG;
  unsigned __int128 v = (((unsigned __int128)f + n) << (l + 1));
  if (v >> 64) return SIEVE_E_RANGE;
  *B = isqrt_u64((uint64_t)v);
  return SIEVE_OK;
}

const char* sieve_strerror(int st) {
  switch (st) {
    case SIEVE_OK: return "ok";
    case SIEVE_E_ARG: return "invalid argument";
    case SIEVE_E_RANGE: return "interval end v does not fit in 64 bits";
    case SIEVE_E_BOUND: return "sieving bound B out of range";
    case SIEVE_E_NOMEM: return "device allocation failed";
    case SIEVE_E_HIP: return "HIP runtime error";
    case SIEVE_E_BUDGET: return "batch exceeds the byte budget";
    case SIEVE_E_DEVICE: return "device kernel reported a violated invariant";
    case SIEVE_E_SCRATCH: return "request exceeds the static scratch of the allocation-free entry point";
    default: return "unknown status";
  }
}

int sieve_last_hip_error(void) { return g_last_hip; }

int sieve_check_device_errors(sieve_ctx* ctx) {
  if (!ctx) return SIEVE_E_ARG;
  std::lock_guard<std::mutex> g(ctx->mu);
  if (!ctx->err_ready) return SIEVE_OK;
  uint32_t v = 0;
  if (ctx->has_last) HIPCHK(hipStreamSynchronize(ctx->last_stream));
  HIPCHK(hipMemcpy(&v, ctx->err.p, 4, hipMemcpyDeviceToHost));
  if (v) {
    uint32_t z = 0;
    HIPCHK(hipMemcpy(ctx->err.p, &z, 4, hipMemcpyHostToDevice));
    return SIEVE_E_DEVICE;
  }
  return SIEVE_OK;
}

int sieve_ctx_set_timing(sieve_ctx* ctx, int enable) {
  if (!ctx) return SIEVE_E_ARG;
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->timing = enable != 0;
  if (!enable) { ctx->times.clear(); }
  return SIEVE_OK;
}

int sieve_ctx_kernel_times(sieve_ctx* ctx, char (*names)[48], double* total_ms, uint64_t* launches, uint32_t cap,
                           uint32_t* count) {
  if (!ctx || !count) return SIEVE_E_ARG;
  std::lock_guard<std::mutex> g(ctx->mu);
  STCHK(collect_times(ctx));
  uint32_t i = 0;
  for (auto& kv : ctx->times) {
    if (i < cap) {
      if (names) { strncpy(names[i], kv.first.c_str(), 47); names[i][47] = 0; }
      if (total_ms) total_ms[i] = kv.second.ms;
      if (launches) launches[i] = kv.second.n;
    }
    ++i;
  }
  *count = i;
  ctx->times.clear();
  return SIEVE_OK;
}

int sieve_copy_calibration(const void* src_dev, void* dst_dev, uint64_t nbytes, void* stream) {
  if (!src_dev || !dst_dev || (nbytes % 16)) return SIEVE_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  sv::k_copy16<<<2048, 256, 0, s>>>((const uint4*)src_dev, (uint4*)dst_dev, nbytes / 16);
  HIPCHK(hipGetLastError());
  return SIEVE_OK;
}

int sieve_microbench(uint32_t kind, uint32_t rounds, double* ops_per_s, void* stream) {
  if (!ops_per_s || kind > SIEVE_MB_MOD64 || rounds == 0 || rounds > (1u << 20)) return SIEVE_E_ARG;
  sieve_ctx* c = sieve_default_ctx();
  if (!c) return SIEVE_E_HIP;
  std::lock_guard<std::mutex> g(c->mu);
  hipStream_t s = (hipStream_t)stream;
  STCHK(begin(c, s));
  STCHK(c->mb_sink.ensure(256));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return SIEVE_E_HIP; }
  double ops = 0;
  hipError_t e = hipEventRecord(e0, s);
  if (e == hipSuccess) {
    if (kind == SIEVE_MB_MOD64) {
      const uint32_t grid = 8 * c->ncu;
      sv::k_mb_mod64<<<grid, 256, 0, s>>>(rounds, 12345u, c->mb_sink.as<uint32_t>());
      ops = (double)grid * 256.0 * rounds * sv::kMbModChains;
    } else if (kind == SIEVE_MB_VALU) {
      const uint32_t grid = 8 * c->ncu;                        // eight waves per SIMD
      sv::k_mb_valu<<<grid, 256, 0, s>>>(rounds, 12345u, c->mb_sink.as<uint32_t>());
      ops = (double)grid * 256.0 * rounds * sv::kMbChains * 2.0;
    } else {
      const uint32_t grid = 4 * c->ncu;                        // four rounds of one workgroup per CU
      sv::k_mb_lds<<<grid, 1024, 0, s>>>(kind == SIEVE_MB_LDS_OR_SPREAD ? 1u : 0u, rounds, 12345u,
                                         c->mb_sink.as<uint32_t>());
      ops = (double)grid * 1024.0 * rounds * sv::kMbAddrs;
    }
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) { g_last_hip = (int)e; return SIEVE_E_HIP; }
  *ops_per_s = ms > 0 ? ops / (1e-3 * ms) : 0.0;
  return end(c, s);
}

int sieve_debug_buckets(uint32_t l, uint64_t f, uint64_t n, uint64_t B, const sieve_tune* tune,
                        uint32_t* bin_start_host, uint32_t bin_cap, uint32_t* entries_host, uint64_t entry_cap,
                        uint32_t* nbins_out, uint32_t* bin_log2, uint64_t* chunk_bits, uint64_t* nlarge,
                        uint64_t* nentries, uint32_t* pad_per_bin) {
  uint64_t F, NB;
  STCHK(check_interval(l, f, n, B, &F, &NB));
  Resolved R;
  STCHK(resolve_tune(l, tune, &R));
  if (!bin_start_host || !nbins_out) return SIEVE_E_ARG;
  const uint64_t med_lim = 1ull << R.Mlog;
  if (B < med_lim) return SIEVE_E_ARG;  // no large primes
  sieve_ctx* c = sieve_default_ctx();
  if (!c) return SIEVE_E_HIP;
  std::lock_guard<std::mutex> g(c->mu);
  hipStream_t s = nullptr;
  STCHK(begin(c, s));
  STCHK(build_primes(c, B, &c->own, s));
  const uint64_t tab_ub = pi_upper(B);
  STCHK(c->plan.ensure(sizeof(sv::Plan) * 2));
  sv::Plan* plan = c->plan.as<sv::Plan>();
  sv::k_plan<<<1, 64, 0, s>>>(c->own.P.as<uint32_t>(), c->own.cnt.as<uint32_t>(), B, 17, 1ull << R.Wlog,
                             1ull << R.Blog, med_lim, 1ull << (R.L - 3), (uint32_t)tab_ub, plan);
  STCHK(c->Q0.ensure(tab_ub * 8 + 64));
  STCHK(c->OFF.ensure(2 * tab_ub * 4 + 64));
  const uint64_t lbits = std::min<uint64_t>(kLaunchBits, NB);
  sv::k_offsets<<<(uint32_t)((tab_ub + 256 * sv::kOffPer - 1) / (256 * sv::kOffPer)), 256, 0, s>>>(c->own.P.as<uint32_t>(), plan, F, lbits,
                                                                 c->Q0.as<uint2>(), c->OFF.as<uint32_t>(), 0);
  const uint32_t b = R.b, esz = b <= 16 ? 2 : 4;
  const uint64_t cbits = std::min<uint64_t>(std::min<uint64_t>((1ull << R.binslog) << b, kLaunchBits), lbits);
  const uint32_t nbins = (uint32_t)((cbits + (1ull << b) - 1) >> b);
  c->h_jobs.clear(); c->h_blk2job.clear(); c->h_cjobs.clear(); c->h_cblk2job.clear(); c->h_thr.clear();
  uint64_t hg = 0;
  chunk_jobs(nbins, (uint32_t)cbits, b, R.R, R.groups, (double)med_lim, (double)B, c->own.P.as<uint32_t>(), plan,
             c->OFF.as<uint32_t>(), c->OFF.as<uint32_t>() + tab_ub, 0, &c->h_jobs, &c->h_blk2job, &c->h_cjobs,
             &c->h_cblk2job, &c->h_thr, &hg);
  uint32_t max_rbins = 1;
  for (auto& J : c->h_jobs) max_rbins = std::max(max_rbins, J.rbins);
  STCHK(c->HG.ensure(hg * 4 + 64));
  STCHK(c->bstart.ensure((2 * nbins + 2) * 4));
  uint32_t lds = 0, pad_bin = 0;
  const uint64_t pad = set_stages(c->h_jobs, 0, c->h_jobs.size(), esz, &lds);
  for (auto& J : c->h_jobs) pad_bin = std::max(pad_bin, J.GR * (sv::kRegionBytes / esz - 1));
  const double rs = recip_sum_upper((double)med_lim, (double)B);
  const uint64_t cap = (uint64_t)(1.02 * rs * (double)cbits) + tab_ub + 4096 + pad;
  if (cap >= 0xFFFFFFFFull) return SIEVE_E_NOMEM;
  STCHK(c->bucket.ensure(cap * esz));
  STCHK(ensure_err(c, s));
  STCHK(pin_begin(c, job_upload_bytes(c)));
  STCHK(upload_jobs(c, s));
  STCHK(pin_end(c, s));
  (void)max_rbins;
  STCHK(bucket_fill_jobs(c, c->jobs.as<sv::BucketJob>(), c->blk2job.as<uint32_t>(), (uint32_t)c->h_jobs.size(),
                         (uint32_t)c->h_blk2job.size(), c->cjobs.as<sv::BucketJob>(), c->cblk2job.as<uint32_t>(),
                         (uint32_t)c->h_cblk2job.size(), nbins, nbins, lds, esz, (uint32_t)cap, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<uint32_t> bs(nbins + 1);
  HIPCHK(hipMemcpy(bs.data(), c->bstart.p, (nbins + 1) * 4, hipMemcpyDeviceToHost));
  sv::Plan hp;
  HIPCHK(hipMemcpy(&hp, plan, sizeof hp, hipMemcpyDeviceToHost));
  *nbins_out = nbins;
  if (bin_log2) *bin_log2 = b;
  if (chunk_bits) *chunk_bits = cbits;
  if (nlarge) *nlarge = hp.np - hp.iM;
  if (nentries) *nentries = bs[nbins];
  if (pad_per_bin) *pad_per_bin = pad_bin;
  memcpy(bin_start_host, bs.data(), std::min<uint32_t>(bin_cap, nbins + 1) * 4);
  if (entries_host) {
    const uint64_t ne = std::min<uint64_t>(std::min<uint64_t>(entry_cap, bs[nbins]), cap);
    if (esz == 4) {
      if (ne) HIPCHK(hipMemcpy(entries_host, c->bucket.p, ne * 4, hipMemcpyDeviceToHost));
    } else {
      std::vector<uint16_t> tmp(ne);
      if (ne) HIPCHK(hipMemcpy(tmp.data(), c->bucket.p, ne * 2, hipMemcpyDeviceToHost));
      for (uint64_t i = 0; i < ne; ++i) entries_host[i] = tmp[i];
    }
  }
  uint32_t ev = 0;
  HIPCHK(hipMemcpy(&ev, c->err.p, 4, hipMemcpyDeviceToHost));
  if (ev) {
    uint32_t z = 0;
    HIPCHK(hipMemcpy(c->err.p, &z, 4, hipMemcpyHostToDevice));
    return SIEVE_E_DEVICE;
  }
  return end(c, s);
}

}  // extern "C"

namespace {

// One window of a batched request (at most kLaunchBits bits).
struct Window {
  uint64_t G0, B;
  uint32_t lbits;
  uint32_t* S;
  uint32_t* counts;
  double cost;
};

int batch_windows(const sieve_primes* pr, uint32_t l, const sieve_req* reqs, size_t nreq, const Resolved& R,
                  std::vector<Window>* out) {
  out->clear();
  for (size_t i = 0; i < nreq; ++i) {
    uint64_t F, NB;
    STCHK(check_interval(l, reqs[i].f, reqs[i].n, reqs[i].B, &F, &NB));
    if (reqs[i].B > pr->B) return SIEVE_E_BOUND;
    if (!reqs[i].S_dev || !reqs[i].counts_dev) return SIEVE_E_ARG;
    for (uint64_t ws = 0; ws < NB; ws += kLaunchBits) {
      Window w;
      w.G0 = F + ws;
      w.B = reqs[i].B;
      w.lbits = (uint32_t)std::min<uint64_t>(kLaunchBits, NB - ws);
      w.S = reqs[i].S_dev + (ws >> 5);
      w.counts = reqs[i].counts_dev + (ws >> l);
      // work estimate: per tile one visit per medium prime, plus the marks
      const double tiles = std::ceil((double)w.lbits / (double)(1u << R.L));
      const double med = (double)pi_upper(std::min<uint64_t>(w.B, 1ull << R.Mlog));
      const double lb = std::log(std::log(std::max<double>((double)w.B, 17.0)));
      w.cost = tiles * med + (double)w.lbits * lb * 0.5;
      out->push_back(w);
    }
  }
  std::stable_sort(out->begin(), out->end(), [](const Window& a, const Window& b) { return a.cost > b.cost; });
  return SIEVE_OK;
}

uint64_t window_cap(const Window& w, uint64_t med_lim) {
  const double rs = recip_sum_upper((double)med_lim, (double)w.B);
  return (uint64_t)(1.02 * rs * (double)w.lbits) + pi_upper(w.B) + 4096;
}

template <typename E>
void launch_tile_batch(uint32_t L, uint32_t grid, hipStream_t s, const sv::BatchReq* rq, uint32_t nreq, uint32_t nitems,
                       const uint2* items, uint32_t* queue, const uint32_t* P, const uint32_t* xpat, const void* bucket,
                       const uint32_t* bstart, uint32_t b, uint32_t cap, uint32_t l, uint32_t* tcnt) {
#define SV_TB(LL)                                                                                                    \
  sv::k_tile_batch<E, LL><<<grid, 1024, 0, s>>>(rq, nreq, nitems, items, queue, P, xpat, bucket, bstart, b, cap, \
                                                l, tcnt)
  switch (L) {
    case 13: SV_TB(13); break;
    case 14: SV_TB(14); break;
    case 15: SV_TB(15); break;
    case 16: SV_TB(16); break;
    case 17: SV_TB(17); break;
    case 18: SV_TB(18); break;
    case 19: SV_TB(19); break;
    default: SV_TB(20); break;
  }
#undef SV_TB
}

}  // namespace

extern "C" {

int sieve_batch(sieve_ctx* ctx, const sieve_primes* pr, uint32_t l, const sieve_req* reqs, size_t nreq,
                const sieve_tune* tune, void* stream) {
  if (!ctx || !pr || (!reqs && nreq)) return SIEVE_E_ARG;
  Resolved R;
  STCHK(resolve_tune(l, tune, &R));
  std::vector<Window> W;
  STCHK(batch_windows(pr, l, reqs, nreq, R, &W));
  if (W.empty()) return SIEVE_OK;
  std::lock_guard<std::mutex> g(ctx->mu);
  sieve_ctx* c = ctx;
  hipStream_t s = (hipStream_t)stream;
  STCHK(begin(c, s));
  const uint32_t L = R.L, b = R.b, esz = b <= 16 ? 2 : 4;
  const uint64_t med_lim = 1ull << R.Mlog;
  const uint32_t nw = (uint32_t)W.size();
  // per-window layout
  c->h_req.assign(nw, sv::BatchReq());
  c->h_blk.clear();
  c->h_seg0.assign(nw, 0);
  uint64_t qp_tot = 0, off_tot = 0, cap_tot = 0, hg_tot = 0;
  uint32_t items = 0, gbins = 0, tcnt = 0, seg_tot = 0, max_rbins = 1;
  const uint32_t* xpat = nullptr;
  const bool seg_long = L < l;
  // work items: runs of consecutive tiles of one request carry offsets from tile to
  // tile (a run's first tile computes every first hit), so early items are long;
  // the queue is taken in order and an item's length shrinks with the tiles still
  // to be claimed (remaining / (2 x resident workgroups), at most kBatchRunMax), so
  // the last items are single tiles and the workgroups finish together
  uint64_t all_tiles = 0;
  for (const Window& X : W) all_tiles += (X.lbits + (1ull << L) - 1) >> L;
  const uint64_t resident = (uint64_t)c->ncu * tiles_per_cu(L);
  c->h_items.clear();
  uint64_t remaining = all_tiles;
  for (uint32_t w = 0; w < nw; ++w) {
    const Window& X = W[w];
    sv::BatchReq& q = c->h_req[w];
    memset(&q, 0, sizeof q);
    q.G0 = X.G0; q.B = X.B; q.lbits = X.lbits;
    q.ntiles = (X.lbits + (1u << L) - 1) >> L;
    q.item0 = items;
    for (uint32_t t = 0; t < q.ntiles;) {
      const uint32_t sz = (uint32_t)std::min<uint64_t>(
          std::min<uint64_t>(kBatchRunMax, std::max<uint64_t>(1, remaining / (2 * resident))), q.ntiles - t);
      c->h_items.push_back(make_uint2(w, t | (sz << 18)));     // t < 2^18 (2^31-bit windows, tiles >= 2^13)
      t += sz;
      remaining -= sz;
    }
    items = (uint32_t)c->h_items.size();
    q.psq = (uint32_t)std::min<uint64_t>(isqrt_u64(2 * X.G0 + 1), 0xFFFFFFFFull);
    const uint32_t* pat; uint32_t per, patw, pmask;
    STCHK(get_pattern(c, X.B, s, &pat, &per, &patw, &pmask));
    q.pat = pat; q.per = per; q.patw = patw; q.per_G0 = (uint32_t)(X.G0 % per);
    q.per_tile = (uint32_t)((1ull << L) % per); q.fixmask = pmask;
    q.xon = use_xpat(X.B, L, l) ? 1u : 0u;
    if (q.xon && !xpat) STCHK(get_xpattern(c, s, &xpat));
    q.qp_cap = (uint32_t)(pi_upper(std::min<uint64_t>(X.B, med_lim)) + 16);
    q.off_cap = (uint32_t)(pi_upper(X.B) + 16);
    q.QP = reinterpret_cast<uint2*>(qp_tot);       // offsets into the slabs; rebased below
    q.OFF = reinterpret_cast<uint32_t*>(off_tot);
    qp_tot += q.qp_cap; off_tot += q.off_cap;
    q.S = X.S; q.counts = X.counts;
    q.tcnt_base = tcnt;
    if (seg_long) tcnt += q.ntiles;
    c->h_seg0[w] = seg_tot;
    seg_tot += X.lbits >> l;
    for (uint32_t k = 0; k * 256u * sv::kOffPer < q.off_cap; ++k) c->h_blk.push_back(make_uint2(w, k));
    if (X.B >= med_lim) {
      q.nbins = (X.lbits + (1u << b) - 1) >> b;
      q.bin_base = gbins;
      gbins += q.nbins;
      cap_tot += window_cap(X, med_lim);
    }
  }
  // bucket jobs: workgroups shared out by estimated work (hits + primes)
  std::vector<double> work(nw, 0.0);
  double work_tot = 0;
  for (uint32_t w = 0; w < nw; ++w) {
    const sv::BatchReq& q = c->h_req[w];
    if (!q.nbins) continue;
    const double hits = recip_sum_upper((double)med_lim, (double)q.B) * q.lbits;
    work[w] = hits + 2.0 * (double)pi_upper(q.B);
    work_tot += work[w];
  }
  c->h_jobs.clear(); c->h_blk2job.clear(); c->h_cjobs.clear(); c->h_cblk2job.clear(); c->h_thr.clear();
  uint32_t max_cbins = 1;
  for (uint32_t w = 0; w < nw; ++w) {
    const sv::BatchReq& q = c->h_req[w];
    if (!q.nbins) continue;
    const uint32_t groups = (uint32_t)std::min<double>((double)R.groups,
                                                       std::max<double>(1.0, std::round((double)R.groups * 2 * work[w] / work_tot)));
    const size_t jb = c->h_jobs.size();
    chunk_jobs(q.nbins, q.lbits, b, R.R, groups, (double)med_lim, (double)q.B, pr->P.as<uint32_t>(),
               reinterpret_cast<const sv::Plan*>((uintptr_t)w), reinterpret_cast<const uint32_t*>((uintptr_t)w), nullptr,
               q.bin_base, &c->h_jobs, &c->h_blk2job, &c->h_cjobs, &c->h_cblk2job, &c->h_thr, &hg_tot);
    for (size_t k = jb; k < c->h_jobs.size(); ++k) max_rbins = std::max(max_rbins, c->h_jobs[k].rbins);
    max_cbins = std::max(max_cbins, q.nbins);
  }
  if (max_rbins > sv::kMaxStageBins || max_cbins > kMaxCountBins) return SIEVE_E_NOMEM;
  uint32_t lds = 0;
  cap_tot += set_stages(c->h_jobs, 0, c->h_jobs.size(), esz, &lds);
  if (cap_tot >= 0xFFFFFFFFull || hg_tot >= 0xFFFFFFFFull) return SIEVE_E_NOMEM;
  // device buffers
  STCHK(c->Q0.ensure(qp_tot * 8 + 64));
  STCHK(c->OFF.ensure(off_tot * 4 + 64));
  STCHK(ensure_err(c, s));
  STCHK(c->b_req.ensure(nw * sizeof(sv::BatchReq)));
  STCHK(c->b_blk.ensure(c->h_blk.size() * sizeof(uint2)));
  STCHK(c->b_seg0.ensure(nw * 4));
  STCHK(c->b_queue.ensure(64));
  STCHK(c->b_items.ensure(c->h_items.size() * sizeof(uint2) + 64));
  if (seg_long) STCHK(c->b_tcnt.ensure((size_t)tcnt * 4 + 64));
  sv::BatchReq* dreq = c->b_req.as<sv::BatchReq>();
  for (sv::BatchReq& q : c->h_req) {
    q.QP = c->Q0.as<uint2>() + reinterpret_cast<uintptr_t>(q.QP);
    q.OFF = c->OFF.as<uint32_t>() + reinterpret_cast<uintptr_t>(q.OFF);
  }
  for (auto* list : {&c->h_jobs, &c->h_cjobs})
    for (sv::BucketJob& J : *list) {   // one chunk per request: no next-chunk offsets
      const uintptr_t w = reinterpret_cast<uintptr_t>(J.plan);
      J.plan = &dreq[w].plan;
      J.OFF_in = c->h_req[w].OFF;
      J.OFF_out = nullptr;
      J.update = 0;
    }
  const uint32_t njobs = (uint32_t)c->h_jobs.size();
  STCHK(pin_begin(c, pad256(nw * sizeof(sv::BatchReq)) + pad256(c->h_blk.size() * sizeof(uint2)) + pad256(nw * 4) +
                         pad256(c->h_items.size() * sizeof(uint2)) + job_upload_bytes(c)));
  STCHK(upload(c, s, c->b_req.p, c->h_req.data(), nw * sizeof(sv::BatchReq)));
  STCHK(upload(c, s, c->b_items.p, c->h_items.data(), c->h_items.size() * sizeof(uint2)));
  STCHK(upload(c, s, c->b_blk.p, c->h_blk.data(), c->h_blk.size() * sizeof(uint2)));
  STCHK(upload(c, s, c->b_seg0.p, c->h_seg0.data(), nw * 4));
  if (njobs) STCHK(upload_jobs(c, s));
  STCHK(pin_end(c, s));
  STCHK(launch(c, "k_fill_u32", s, [&] { sv::k_fill_u32<<<1, 64, 0, s>>>(c->b_queue.as<uint32_t>(), 16, 0); }));
  STCHK(launch(c, "k_plan_batch", s, [&] {
    sv::k_plan_batch<<<(nw + 63) / 64, 64, 0, s>>>(pr->P.as<uint32_t>(), pr->cnt.as<uint32_t>(), dreq, nw,
                                                   1ull << R.Wlog, 1ull << R.Blog, med_lim, 1ull << (L - 3));
  }));
  const uint32_t nblk = (uint32_t)c->h_blk.size();
  STCHK(launch(c, "k_offsets_batch", s, [&] {
    sv::k_offsets_batch<<<nblk, 256, 0, s>>>(pr->P.as<uint32_t>(), dreq, c->b_blk.as<uint2>());
  }));
  uint32_t cap32 = 0;
  if (njobs) {
    STCHK(c->HG.ensure(hg_tot * 4 + 64));
    STCHK(c->bstart.ensure(((size_t)2 * gbins + 2) * 4));
    STCHK(c->bucket.ensure(cap_tot * esz));
    cap32 = (uint32_t)cap_tot;
    STCHK(bucket_fill_jobs(c, c->jobs.as<sv::BucketJob>(), c->blk2job.as<uint32_t>(), njobs,
                           (uint32_t)c->h_blk2job.size(), c->cjobs.as<sv::BucketJob>(), c->cblk2job.as<uint32_t>(),
                           (uint32_t)c->h_cblk2job.size(), max_cbins, gbins, lds, esz, cap32, s));
  }
  int ncu = 0;
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device));
  const uint32_t grid = (uint32_t)std::min<uint64_t>((uint64_t)ncu * tiles_per_cu(L), items);
  uint32_t* tc = seg_long ? c->b_tcnt.as<uint32_t>() : nullptr;
  const void* bk = njobs ? c->bucket.p : nullptr;
  const uint32_t* bsp = njobs ? c->bstart.as<uint32_t>() : nullptr;
  if (esz == 2)
    STCHK(launch(c, "k_tile_batch", s, [&] {
      launch_tile_batch<uint16_t>(L, grid, s, dreq, nw, items, c->b_items.as<uint2>(), c->b_queue.as<uint32_t>(), pr->P.as<uint32_t>(), xpat, bk, bsp,
                                  b, cap32, l, tc);
    }));
  else
    STCHK(launch(c, "k_tile_batch", s, [&] {
      launch_tile_batch<uint32_t>(L, grid, s, dreq, nw, items, c->b_items.as<uint2>(), c->b_queue.as<uint32_t>(), pr->P.as<uint32_t>(), xpat, bk, bsp,
                                  b, cap32, l, tc);
    }));
  if (seg_long)
    STCHK(launch(c, "k_counts_batch", s, [&] {
      sv::k_counts_batch<<<(seg_tot + 255) / 256, 256, 0, s>>>(dreq, nw, c->b_seg0.as<uint32_t>(), seg_tot, tc, l - L);
    }));
  return end(c, s);
}

int sieve_batch_scratch_bytes(const sieve_primes* pr, uint32_t l, const sieve_req* reqs, size_t nreq,
                              const sieve_tune* tune, uint64_t* bytes) {
  if (!pr || !bytes || (!reqs && nreq)) return SIEVE_E_ARG;
  std::vector<sieve_req> rr(reqs, reqs + nreq);
  for (auto& r : rr) { if (!r.S_dev) r.S_dev = reinterpret_cast<uint32_t*>(16); if (!r.counts_dev) r.counts_dev = reinterpret_cast<uint32_t*>(16); }
  return dry_bytes([&](sieve_ctx* c) { return sieve_batch(c, pr, l, rr.data(), nreq, tune, nullptr); }, bytes);
}

int sieve_sieve_scratch_bytes(const sieve_primes* pr, uint32_t l, uint64_t f, uint64_t n, uint64_t B,
                              const sieve_tune* tune, uint64_t* bytes) {
  if (!bytes) return SIEVE_E_ARG;
  uint32_t* dummy = reinterpret_cast<uint32_t*>(16);
  return dry_bytes([&](sieve_ctx* c) {
    return pr ? sieve_ctx_sieve_with(c, pr, l, f, n, B, dummy, dummy, tune, nullptr)
              : sieve_ctx_sieve(c, l, f, n, B, dummy, dummy, tune, nullptr);
  }, bytes);
}

int sieve_ctx_scratch_bytes(sieve_ctx* ctx, uint64_t* bytes) {
  if (!ctx || !bytes) return SIEVE_E_ARG;
  std::lock_guard<std::mutex> g(ctx->mu);
  uint64_t tot = 0;
  ctx->each_buf([&](DevBuf& b) { if (!b.fixed) tot += b.bytes; });
  *bytes = tot;
  return SIEVE_OK;
}

int sieve_ctx_trim(sieve_ctx* ctx) {
  if (!ctx) return SIEVE_E_ARG;
  std::lock_guard<std::mutex> g(ctx->mu);
  if (ctx->has_last) HIPCHK(hipStreamSynchronize(ctx->last_stream));
  ctx->each_buf([](DevBuf& b) { b.release(); });
  for (auto& w : ctx->pat_words) w = 0;
  ctx->xpat_ready = false;
  ctx->err_ready = false;
  return SIEVE_OK;
}

int sieve_primes_bytes(const sieve_primes* pr, uint64_t* bytes) {
  if (!pr || !bytes) return SIEVE_E_ARG;
  *bytes = pr->P.bytes + pr->cnt.bytes;
  return SIEVE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free variant of sieve_init.  Its scratch (prime table, generator
// table, plan, first offsets, patterns, error word) lives in one static device
// array; the host reaches it only through the address hipGetSymbolAddress
// returns for the current device.  It serves the requests whose sieving primes
// all stay in LDS (B below the default medium bound 2^tile_log2, so no buckets)
// and whose table fits one tile launch (at most four 2^31-bit windows); every
// such request fits the array below.
namespace {

constexpr size_t kScratchBytes = (size_t)4 << 20;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

struct NoAllocDev {
  sieve_ctx* ctx = nullptr;        // its DevBufs are fixed slices of the device's scratch
  unsigned char* base = nullptr;   // device address of scratch on this device
};
std::mutex g_na_mu;
NoAllocDev g_na[kMaxDevices];

// Largest bound and window count the scratch is laid out for.
constexpr uint64_t kNaMaxB = (1ull << 20) - 1;

// Carves the fixed buffers of ctx out of [base, base + kScratchBytes); returns
// SIEVE_E_SCRATCH if the layout does not fit (a build-time constant mistake).
int carve_noalloc(sieve_ctx* c, unsigned char* base) {
  size_t off = 0;
  bool ok = true;
  auto take = [&](DevBuf& b, size_t n) {
    off = (off + 255) & ~size_t(255);
    b.p = base + off;
    b.bytes = n;
    b.fixed = true;
    off += n;
    if (off > kScratchBytes) ok = false;
  };
  const uint64_t tab_ub = pi_upper(kNaMaxB);
  const uint64_t base_ub = pi_upper(65536);
  take(c->own.P, (size_t)(tab_ub + 16) * 4);
  take(c->own.cnt, 16);
  take(c->gen_blk, (size_t)base_ub * 4 + 64);
  take(c->plan, sizeof(sv::Plan) * 2);
  // generator offsets, then every window's medium-prime offsets of the tile launch
  take(c->Q0, std::max<size_t>((size_t)base_ub * 8, (size_t)sv::kMaxWins * tab_ub * 8 + 64));
  const uint64_t gbits = 1ull << 19;   // odd numbers below 2^20, whole 2^15-bit count segments
  const uint64_t nwords = gbits / 32;
  take(c->gen_S, (size_t)(nwords + (nwords + 1023) / 1024 + (gbits >> 15) + 64) * 4);
  take(c->err, 64);
  for (auto& b : c->pat) take(b, (size_t)sv::kPatWordsMax * 4);
  take(c->xpat, (size_t)sv::kXWordsAll * 4);
  return ok ? SIEVE_OK : SIEVE_E_SCRATCH;
}

// Set-up on the first call on a device (that device current): the scratch's
// device address and a context whose buffers are slices of it.
int noalloc_setup(int dev, sieve_ctx** out) {
  std::lock_guard<std::mutex> g(g_na_mu);
  NoAllocDev& d = g_na[dev];
  if (!d.ctx) {
    unsigned char* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)));
    sieve_ctx* c = new (std::nothrow) sieve_ctx();
    if (!c) return SIEVE_E_NOMEM;
    const int rc = carve_noalloc(c, ptr);
    if (rc != SIEVE_OK) { delete c; return rc; }
    d.base = ptr;
    d.ctx = c;
  }
  *out = d.ctx;
  return SIEVE_OK;
}

}  // namespace

extern "C" int sieve_init_noalloc(uint32_t l, uint64_t f, uint64_t n, uint64_t B, uint32_t* S_dev,
                                  uint32_t* counts_dev, void* stream) {
  // argument and size checks come before any HIP call
  if (!S_dev || !counts_dev) return SIEVE_E_ARG;
  uint64_t F, NB;
  STCHK(check_interval(l, f, n, B, &F, &NB));
  Resolved R;
  STCHK(resolve_tune(l, nullptr, &R));
  if (B >= (1ull << R.Mlog) || B > kNaMaxB) return SIEVE_E_SCRATCH;             // no bucket path
  if ((NB + kLaunchBits - 1) / kLaunchBits > sv::kMaxWins) return SIEVE_E_SCRATCH;   // one tile launch
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return SIEVE_E_ARG;
  sieve_ctx* c = nullptr;
  STCHK(noalloc_setup(dev, &c));
  std::lock_guard<std::mutex> g(c->mu);
  hipStream_t s = (hipStream_t)stream;
  STCHK(begin(c, s));
  STCHK(build_primes(c, B, &c->own, s));
  STCHK(run_sieve(c, &c->own, l, F, NB, B, S_dev, counts_dev, R, s));
  return end(c, s);
}

extern "C" int sieve_goldbach(sieve_ctx* ctx, const sieve_primes* pr, uint32_t l, uint64_t f, uint64_t n,
                              const uint32_t* S_dev, uint64_t Q, uint32_t* maxq_dev, uint64_t* argk_dev,
                              uint32_t* fails_dev, uint32_t* minq_dev, void* stream) {
  if (!ctx || !pr || !S_dev || !maxq_dev || !argk_dev || !fails_dev) return SIEVE_E_ARG;
  uint64_t F, NB;
  STCHK(check_interval(l, f, n, 3, &F, &NB));
  if (Q < 3 || Q > pr->B) return SIEVE_E_BOUND;
  if ((NB / 32 + 255) / 256 > 0x7FFFFFFFull) return SIEVE_E_ARG;
  std::lock_guard<std::mutex> g(ctx->mu);
  sieve_ctx* c = ctx;
  hipStream_t s = (hipStream_t)stream;
  STCHK(begin(c, s));
  STCHK(c->gb_best.ensure((size_t)n * 8 + 64));
  STCHK(c->gb_k.ensure(64));
  unsigned long long* best = c->gb_best.as<unsigned long long>();
  const uint32_t fill_blocks = (uint32_t)std::min<uint64_t>((2 * n + 255) / 256, 4096);
  STCHK(launch(c, "k_fill_u32", s, [&] { sv::k_fill_u32<<<fill_blocks, 256, 0, s>>>(c->gb_best.as<uint32_t>(), 2 * n, 0); }));
  STCHK(launch(c, "k_fill_u32", s, [&] {
    sv::k_fill_u32<<<(uint32_t)std::min<uint64_t>((n + 255) / 256, 4096), 256, 0, s>>>(fails_dev, n, 0);
  }));
  if (minq_dev)
    STCHK(launch(c, "k_fill_u32", s, [&] { sv::k_fill_u32<<<4096, 256, 0, s>>>(minq_dev, NB, 0); }));
  STCHK(launch(c, "k_gb_count", s, [&] {
    sv::k_gb_count<<<1, 1, 0, s>>>(pr->P.as<uint32_t>(), pr->cnt.as<uint32_t>(), Q, c->gb_k.as<uint32_t>());
  }));
  sv::GbArgs a;
  a.S = S_dev; a.nwords = NB / 32; a.P = pr->P.as<uint32_t>(); a.K = c->gb_k.as<uint32_t>(); a.l = l;
  a.best = best; a.fails = fails_dev; a.minq = minq_dev;
  const uint64_t grid = (a.nwords + 255) / 256;
  STCHK(launch(c, "k_goldbach", s, [&] {
    if (minq_dev) sv::k_goldbach<true><<<(uint32_t)grid, 256, 0, s>>>(a);
    else sv::k_goldbach<false><<<(uint32_t)grid, 256, 0, s>>>(a);
  }));
  STCHK(launch(c, "k_gb_finish", s, [&] {
    sv::k_gb_finish<<<(uint32_t)((n + 255) / 256), 256, 0, s>>>(best, n, l, maxq_dev, argk_dev);
  }));
  return end(c, s);
}

extern "C" int sieve_logsieve(sieve_ctx* ctx, const sieve_primes* pr, uint32_t l, uint64_t f, uint64_t n, uint64_t B,
                              uint32_t T, uint32_t* C_dev, uint32_t* counts_dev, uint8_t* A_dev,
                              const sieve_tune* tune, void* stream) {
  if (!ctx || !C_dev || !counts_dev || T > 255) return SIEVE_E_ARG;
  uint64_t F, NB;
  STCHK(check_interval(l, f, n, B, &F, &NB));
  if (pr && B > pr->B) return SIEVE_E_BOUND;
  // defaults measured on 2^32 positions at 1e12 with the primes up to 2^20: tiles of
  // 2^17 positions, four bin ranges of 256 fill workgroups each (7.7 ms; 10.4 ms with
  // 2^16-position tiles, two ranges and 2048 workgroups per range)
  const uint32_t L = tune && tune->tile_log2 ? tune->tile_log2 : 17;
  if (L < 14 || L > 17) return SIEVE_E_ARG;
  const uint32_t groups = tune && tune->groups ? tune->groups : 1024;
  const uint32_t ranges = tune && tune->ranges ? tune->ranges : 4;
  if (groups < 64 || groups > 4096 || (ranges != 0 && ranges != 1 && ranges != 2 && ranges != 4 && ranges != 8))
    return SIEVE_E_ARG;
  std::lock_guard<std::mutex> g(ctx->mu);
  hipStream_t s = (hipStream_t)stream;
  STCHK(begin(ctx, s));
  if (!pr) {
    STCHK(build_primes(ctx, B, &ctx->own, s));
    pr = &ctx->own;
  }
  STCHK(run_logsieve(ctx, pr, l, F, NB, B, T, C_dev, counts_dev, A_dev, L, groups, ranges, s));
  return end(ctx, s);
}

// Intervals beyond 2^64 (Section 5 names sieving with primes of up to 64 bits as
// the extension of the 32-bit implementation).  The 32-bit primes take the
// ordinary path with 128-bit first offsets; the primes above 2^32 are produced a
// slice at a time by sieving the odd numbers above 2^32 (with the primes up to the
// slice's square root, Section 1.4) and mark the table directly; the counts are
// then taken again.
namespace {
constexpr uint64_t kWideMaxB = 1ull << 40;
constexpr uint32_t kSliceLog = 20;                // segment size of a slice sieve
constexpr uint64_t kSliceBits = 1ull << 30;       // odd numbers per slice
// 3*5*7*...*47: the tile kernel reads the start of the interval only modulo the
// pattern periods (divisors of 3*5*7*11*13 and of 17*19*23, 29*31*37, 41*43*47)
constexpr uint64_t kProxyMod = 307444891294245705ull;
constexpr double kWideListMin = 96.0;       // fewest expected hits per workgroup for the list mode
constexpr double kWideSortHits = 7600.0;    // expected hits per sorting workgroup (sv::kSpK at most)

int check_wide(uint32_t l, uint64_t f_lo, uint64_t f_hi, uint64_t n, uint64_t B, uint64_t* Flo, uint64_t* Fhi,
               uint64_t* NB) {
  if (l < 5 || l > 20 || n == 0) return SIEVE_E_ARG;
  if (B < 3 || B > kWideMaxB) return SIEVE_E_BOUND;
  if ((n >> (40 - l)) || (n >> 31)) return SIEVE_E_ARG;
  typedef unsigned __int128 u128;
  const u128 f = ((u128)f_hi << 64) | f_lo;
  if (f >> (127 - l)) return SIEVE_E_RANGE;
  const u128 F = f << l, N = (u128)n << l;
  if ((F >> 63) == 0) return SIEVE_E_RANGE;         // u = 2F + 1 below 2^64
  if ((F + N) >> 127) return SIEVE_E_RANGE;         // v = 2(F + NB) not below 2^128
  *Flo = (uint64_t)F; *Fhi = (uint64_t)(F >> 64); *NB = (uint64_t)N;
  return SIEVE_OK;
}
}  // namespace

extern "C" int sieve_wide(sieve_ctx* ctx, uint32_t l, uint64_t f_lo, uint64_t f_hi, uint64_t n, uint64_t B,
                          uint32_t* S_dev, uint32_t* counts_dev, const sieve_tune* tune, void* stream) {
  if (!ctx || !S_dev || !counts_dev) return SIEVE_E_ARG;
  uint64_t W[2], NB;
  STCHK(check_wide(l, f_lo, f_hi, n, B, &W[0], &W[1], &NB));
  const uint32_t wlist = tune ? tune->wide_list : 0u;
  const uint32_t hcap_log = tune && tune->wide_slot_log2 ? tune->wide_slot_log2 : 12u;
  const double sort_hits = tune && tune->wide_sort_hits ? (double)tune->wide_sort_hits : kWideSortHits;
  if (wlist > 2 || hcap_log < 6 || hcap_log > 13 || sort_hits < 16.0 || sort_hits > 65536.0) return SIEVE_E_ARG;
  const uint32_t hcap = 1u << hcap_log;
  Resolved R, Rs;
  STCHK(resolve_tune(l, nullptr, &R));
  STCHK(resolve_tune(kSliceLog, nullptr, &Rs));
  typedef unsigned __int128 u128;
  const uint64_t Fp = kProxyMod + (uint64_t)((((u128)W[1] << 64) | W[0]) % kProxyMod);
  const uint64_t B32 = std::min<uint64_t>(B, 0xFFFFFFFFull);
  std::lock_guard<std::mutex> g(ctx->mu);
  sieve_ctx* c = ctx;
  hipStream_t s = (hipStream_t)stream;
  STCHK(begin(c, s));
  STCHK(build_primes(c, B32, &c->own, s));
  STCHK(run_sieve(c, &c->own, l, Fp, NB, B32, S_dev, counts_dev, R, s, W));
  if (B > 0xFFFFFFFFull) {
    const uint64_t k_lo = 1ull << 31, k_hi = (B - 1) / 2;     // indices of 2^32 + 1 and of the last odd <= B
    const uint64_t need = std::min<uint64_t>(kSliceBits, ((k_hi - k_lo + 1 + (1ull << kSliceLog) - 1) >> kSliceLog) << kSliceLog);
    STCHK(c->wsl.ensure(need / 8 + (need >> kSliceLog) * 4 + 256));
    uint32_t* sl = c->wsl.as<uint32_t>();
    uint32_t* slc = sl + need / 32;
    // The slices, and which of them list their hits for a sort by table range
    // instead of OR-ing them in with atomics: tables of at most 2^31 bits (one hit
    // per prime at most), and slices whose workgroups expect at least kWideListMin
    // hits (65536 odd numbers, prime density 2 / ln p, hit probability NB / p at the
    // slice's smallest p); G slots per sorting workgroup for about kWideSortHits hits.
    struct Slice { uint64_t Fs, NBs; uint32_t nw, g, G, nsort; bool list; };
    std::vector<Slice> slices;
    uint32_t nregions = 0, gmax = 0;
    for (uint64_t Fs = k_lo; Fs <= k_hi; Fs += kSliceBits) {
      Slice z;
      z.Fs = Fs;
      z.NBs = std::min<uint64_t>(need, ((k_hi - Fs + 1 + (1ull << kSliceLog) - 1) >> kSliceLog) << kSliceLog);
      z.nw = (uint32_t)(z.NBs / 32);
      z.g = (z.nw + 256 * sv::kWideRounds - 1) / (256 * sv::kWideRounds);
      const double plo = 2.0 * (double)Fs + 1.0;
      const double e = 256.0 * sv::kWideRounds * 32.0 * (2.0 / std::log(plo)) * std::min(1.0, (double)NB / plo);
      z.list = NB <= kLaunchBits && (wlist == 2 || (wlist == 0 && e >= kWideListMin));
      z.G = z.list ? (uint32_t)std::max(1.0, std::min<double>(sv::kHsMaxG, std::floor(sort_hits / e))) : 0;
      z.nsort = z.list ? ((z.g + z.G - 1) / z.G + 7) / 8 * 8 : 0;
      nregions += z.nsort;
      if (z.list) gmax = std::max(gmax, z.g);
      slices.push_back(z);
    }
    if ((uint64_t)nregions * sv::kSpK >= 0xFFFFFFFFull) {   // region offsets are 32-bit: atomics for all
      for (Slice& z : slices) { z.list = false; z.G = z.nsort = 0; }
      nregions = 0;
    }
    const uint32_t wbin = sp_binlog(NB);
    const uint32_t wnbins = (uint32_t)((NB + (1ull << wbin) - 1) >> wbin);
    if (nregions) {
      STCHK(c->wH.ensure((size_t)gmax * hcap * 4));
      STCHK(c->wHc.ensure((size_t)gmax * 4 + 64));
      STCHK(c->wE.ensure((size_t)nregions * sv::kSpK * 4));
      STCHK(c->wHd.ensure((size_t)nregions * wnbins * 4 + 64));
    }
    uint32_t out0 = 0;
    for (const Slice& z : slices) {
      const uint64_t Fs = z.Fs, NBs = z.NBs;
      const uint64_t Bs = std::max<uint64_t>(3, isqrt_u64(2 * (Fs + NBs)));
      STCHK(run_sieve(c, &c->own, kSliceLog, Fs, NBs, Bs, sl, slc, Rs, s));
      const uint32_t nw = z.nw, g = z.g;
      uint32_t* H = c->wH.as<uint32_t>();
      uint32_t* Hc = c->wHc.as<uint32_t>();
      // remainder digits as wide as p < 2^(53-D) allows: 7, 8 or 11 steps
      STCHK(launch(c, "k_wide_hits", s, [&] {
        if (z.list) {
          if (B <= (1ull << 33)) sv::k_wide_hits<20, true><<<g, 256, 0, s>>>(sl, nw, Fs, B, W[0], W[1], NB, S_dev, H, Hc, hcap);
          else if (B <= (1ull << 36)) sv::k_wide_hits<17, true><<<g, 256, 0, s>>>(sl, nw, Fs, B, W[0], W[1], NB, S_dev, H, Hc, hcap);
          else sv::k_wide_hits<12, true><<<g, 256, 0, s>>>(sl, nw, Fs, B, W[0], W[1], NB, S_dev, H, Hc, hcap);
        } else {
          if (B <= (1ull << 33)) sv::k_wide_hits<20, false><<<g, 256, 0, s>>>(sl, nw, Fs, B, W[0], W[1], NB, S_dev, nullptr, nullptr, 0);
          else if (B <= (1ull << 36)) sv::k_wide_hits<17, false><<<g, 256, 0, s>>>(sl, nw, Fs, B, W[0], W[1], NB, S_dev, nullptr, nullptr, 0);
          else sv::k_wide_hits<12, false><<<g, 256, 0, s>>>(sl, nw, Fs, B, W[0], W[1], NB, S_dev, nullptr, nullptr, 0);
        }
      }));
      if (z.list) {
        STCHK(launch(c, "k_hits_sort", s, [&] {
          sv::k_hits_sort<<<z.nsort, sv::kSpThreads, 0, s>>>(H, Hc, hcap, g, z.G, wbin, wnbins, out0, nregions,
                                                             c->wE.as<uint32_t>(), c->wHd.as<uint32_t>(), S_dev);
        }));
        out0 += z.nsort;
      }
    }
    if (nregions)
      STCHK(launch(c, "k_sparse_apply", s, [&] {
        sv::k_sparse_apply<<<wnbins, sv::kSpApplyThreads, (1u << wbin) / 8, s>>>(
            c->wE.as<uint32_t>(), c->wHd.as<uint32_t>(), nregions, wbin, NB, S_dev);
      }));
    const uint32_t nseg = (uint32_t)n;
    const uint32_t grid = l >= 13 ? nseg : (nseg + 255) / 256;
    STCHK(launch(c, "k_recount", s, [&] { sv::k_recount<<<grid, 256, 0, s>>>(S_dev, l, nseg, counts_dev); }));
  }
  return end(c, s);
}
