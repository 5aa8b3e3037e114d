// Host side of the C ABI declared in include/dode.h: argument checks, device
// copies of the assignment matrices, minibatch schedules and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "dode_internal.h"

namespace {

// clusters of at most this many days use the sparse kernels under kernel_path 0
constexpr int32_t kSparseDays = 2;

}  // namespace

namespace {

thread_local std::string g_err;

dode_status fail(dode_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(e_ == hipErrorOutOfMemory ? DODE_ERR_OOM : DODE_ERR_HIP, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                       \
  } while (0)

inline hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

// Stream-ordered scratch allocation released at scope exit on the same stream.
struct DevBuf {
  void* p = nullptr;
  hipStream_t s = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p) (void)hipFreeAsync(p, s);
  }
  hipError_t alloc(size_t bytes, hipStream_t st) {
    s = st;
    return hipMallocAsync(&p, bytes ? bytes : 16, st);
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

size_t state_size(const dode_dar* d) { return d->storage == DODE_F64 ? 8 : 4; }

dode_status check_dims(const dode_dims* dm) {
  if (!dm) return fail(DODE_ERR_ARG, "dims is NULL");
  if (dm->P < 1 || dm->L < 1 || dm->T < 1 || dm->H < 1 || dm->K < 1)
    return fail(DODE_ERR_SHAPE, "dims must be >= 1 (P=%d L=%d T=%d H=%d K=%d)", dm->P, dm->L,
                dm->T, dm->H, dm->K);
  if (dm->K > 64) return fail(DODE_ERR_SHAPE, "K=%d exceeds 64", dm->K);
  if ((int64_t)dm->T * dm->P > (1LL << 31) || (int64_t)dm->H * dm->L > (1LL << 31))
    return fail(DODE_ERR_SHAPE, "per-day vectors exceed 2^31 entries");
  return DODE_OK;
}

dode_status check_dar(const dode_dar* dar, int32_t cluster) {
  if (!dar) return fail(DODE_ERR_ARG, "dar handle is NULL");
  if (cluster < 0 || cluster >= dar->C)
    return fail(DODE_ERR_ARG, "cluster %d out of range [0, %d)", cluster, dar->C);
  return DODE_OK;
}

dode_status check_days(int32_t n_days) {
  if (n_days < 0) return fail(DODE_ERR_ARG, "n_days=%d is negative", n_days);
  if (n_days > 65535) return fail(DODE_ERR_SHAPE, "n_days=%d exceeds 65535 per call", n_days);
  return DODE_OK;
}

// ------------------------------------------------ permutations / schedule --
uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

struct HostSched {
  int32_t bh = 0, nch = 0, mt = 0;
  std::vector<int32_t> perm, pos, touched;   // [E][C][H], [E][C][H], [E][nch][C][mt]
  // component schedule (CompSched): [E][nch][C][bh], [E][nch][C][mt][K+3],
  // [E][nch][C][max_comp][4]
  int32_t max_comp = 1;
  std::vector<int32_t> kslot, kdesc, kcomp;
  // reached-interval chunks (ChunkList): [E][nch][C][max_chunks][chunk_w]
  int32_t max_chunks = 1, chunk_w = 0;
  std::vector<int32_t> kchunk;
};

// Descriptor of departure interval t for the minibatch at positions
// j0..j0+bh-1 of a permutation with inverse `pos`: [t, lag mask, slot per lag].
void fill_desc(int32_t* dsc, int32_t t, const int32_t* pos, int32_t j0, int32_t bh, int32_t H,
               int32_t K) {
  dsc[kDescT] = t;
  uint64_t mask = 0;
  for (int32_t l = 0; l < K; ++l) {
    const int32_t h = t + l;
    const int32_t sl = h < H ? pos[h] - j0 : -1;
    const bool in = sl >= 0 && sl < bh;
    dsc[kDescSlot + l] = in ? sl : -1;
    if (in) mask |= 1ull << l;
  }
  dsc[kDescMask] = (int32_t)(uint32_t)mask;
  dsc[kDescMask + 1] = (int32_t)(uint32_t)(mask >> 32);
}

// Minibatch layout for epochs of C clusters from permutations perm [E][C][H].
dode_status build_sched(const dode_dims& dm, int32_t C, int32_t E, int32_t bh,
                        const int32_t* perm, uint64_t seed, HostSched& hs) {
  const int32_t H = dm.H, T = dm.T, K = dm.K;
  hs.bh = bh;
  hs.nch = (H + bh - 1) / bh;
  hs.mt = std::min<int32_t>(T, bh * K);
  const size_t ech = (size_t)E * C * H;
  hs.perm.resize(ech);
  hs.pos.assign(ech, -1);
  if (perm) {
    std::memcpy(hs.perm.data(), perm, ech * sizeof(int32_t));
  } else {
    uint64_t s = seed;
    for (size_t ec = 0; ec < (size_t)E * C; ++ec) {
      int32_t* p = hs.perm.data() + ec * H;
      for (int32_t i = 0; i < H; ++i) p[i] = i;
      for (int32_t i = H - 1; i > 0; --i) std::swap(p[i], p[splitmix64(s) % (uint64_t)(i + 1)]);
    }
  }
  for (size_t ec = 0; ec < (size_t)E * C; ++ec) {
    const int32_t* p = hs.perm.data() + ec * H;
    int32_t* q = hs.pos.data() + ec * H;
    for (int32_t i = 0; i < H; ++i) {
      if (p[i] < 0 || p[i] >= H || q[p[i]] >= 0)
        return fail(DODE_ERR_ARG, "perm[%zu][%zu] is not a permutation of 0..H-1", ec / C, ec % C);
      q[p[i]] = i;
    }
  }
  // departure intervals each minibatch reaches, packed to the largest count seen;
  // each entry is a descriptor [t, lag mask (2 words), slot of t+0, ..., slot of
  // t+K-1] (slot = position of interval t+l inside the minibatch, -1 if t+l is
  // not in it; mask bit l set when it is)
  std::vector<int32_t> tl;
  tl.assign((size_t)E * hs.nch * C * hs.mt, -1);
  std::vector<char> mark(T);
  int32_t mt_used = 1;
  for (int32_t e = 0; e < E; ++e)
    for (int32_t c = 0; c < C; ++c) {
      const int32_t* p = hs.perm.data() + ((size_t)e * C + c) * H;
      for (int32_t j = 0; j < hs.nch; ++j) {
        std::fill(mark.begin(), mark.end(), 0);
        for (int32_t s = j * bh; s < std::min(H, (j + 1) * bh); ++s)
          for (int32_t l = 0; l < K; ++l) {
            const int32_t t = p[s] - l;
            if (t >= 0 && t < T) mark[t] = 1;
          }
        int32_t* out = tl.data() + (((size_t)e * hs.nch + j) * C + c) * hs.mt;
        int32_t n = 0;
        for (int32_t t = 0; t < T; ++t)
          if (mark[t]) out[n++] = t;
        mt_used = std::max(mt_used, n);
      }
    }
  const size_t dw = desc_width(K);
  hs.touched.assign((size_t)E * hs.nch * C * mt_used * dw, -1);
  for (int32_t e = 0; e < E; ++e)
    for (int32_t j = 0; j < hs.nch; ++j)
      for (int32_t c = 0; c < C; ++c) {
        const size_t r = ((size_t)e * hs.nch + j) * C + c;
        const int32_t* pos = hs.pos.data() + ((size_t)e * C + c) * H;
        // the n reached intervals are spread evenly over the mt_used entries
        // (padding in between), so any contiguous range of the grouped
        // kernels' items holds its share of useful work
        int32_t n = 0;
        while (n < hs.mt && tl[r * hs.mt + n] >= 0) ++n;
        for (int32_t k = 0; k < n; ++k) {
          const int32_t t = tl[r * hs.mt + k];
          const int32_t i = (int32_t)((int64_t)k * mt_used / n);
          fill_desc(hs.touched.data() + (r * mt_used + i) * dw, t, pos, j * bh, bh, H, K);
        }
      }
  // Components of each minibatch: its intervals sorted, cut where two
  // neighbours are K or more apart.  Component [h_a .. h_b] reaches the
  // departure intervals max(0, h_a-K+1) .. min(T-1, h_b), all of them, and no
  // other component reaches any of these.
  // Each component's reached intervals are also cut into chunks of up to
  // kChunkT consecutive ones, listed with the minibatch intervals (and their
  // slots) that reach them: [t0, n_t, n_h, (h, slot) x n_h].
  std::vector<int32_t> ncomp((size_t)E * hs.nch * C, 0), nchunk((size_t)E * hs.nch * C, 0);
  std::vector<std::pair<int32_t, int32_t>> hsl;
  hs.chunk_w = 3 + 2 * (kChunkT + K - 1);
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      hs.kslot.assign((size_t)E * hs.nch * C * bh, -1);
      hs.kdesc.assign((size_t)E * hs.nch * C * mt_used * dw, -1);
      hs.kcomp.assign((size_t)E * hs.nch * C * hs.max_comp * 4, 0);
      hs.kchunk.assign((size_t)E * hs.nch * C * hs.max_chunks * hs.chunk_w, 0);
    }
    for (int32_t e = 0; e < E; ++e)
      for (int32_t j = 0; j < hs.nch; ++j)
        for (int32_t c = 0; c < C; ++c) {
          const size_t r = ((size_t)e * hs.nch + j) * C + c;
          const int32_t* p = hs.perm.data() + ((size_t)e * C + c) * H;
          const int32_t* pos = hs.pos.data() + ((size_t)e * C + c) * H;
          hsl.clear();
          for (int32_t sl = 0; sl < bh && j * bh + sl < H; ++sl) hsl.push_back({p[j * bh + sl], sl});
          std::sort(hsl.begin(), hsl.end());
          int32_t nc = 0, nd = 0, nk = 0;
          for (size_t a = 0; a < hsl.size();) {
            size_t b = a + 1;
            while (b < hsl.size() && hsl[b].first - hsl[b - 1].first < K) ++b;
            {
              const int32_t tlo = std::max(0, hsl[a].first - K + 1);
              const int32_t thi = std::min(T - 1, hsl[b - 1].first);
              for (int32_t t0 = tlo; t0 <= thi; t0 += kChunkT, ++nk) {
                if (pass == 0) continue;
                const int32_t nt = std::min(kChunkT, thi - t0 + 1);
                int32_t* ck = hs.kchunk.data() + (r * hs.max_chunks + nk) * hs.chunk_w;
                ck[0] = t0;
                ck[1] = nt;
                int32_t nh = 0;
                for (size_t q = a; q < b; ++q)
                  if (hsl[q].first >= t0 && hsl[q].first <= t0 + nt - 1 + K - 1) {
                    ck[3 + 2 * nh] = hsl[q].first;
                    ck[4 + 2 * nh] = hsl[q].second;
                    ++nh;
                  }
                ck[2] = nh;
              }
            }
            if (pass == 1) {
              const int32_t tlo = std::max(0, hsl[a].first - K + 1);
              const int32_t thi = std::min(T - 1, hsl[b - 1].first);
              int32_t* cp = hs.kcomp.data() + (r * hs.max_comp + nc) * 4;
              cp[0] = (int32_t)a;
              cp[1] = (int32_t)(b - a);
              cp[2] = nd;
              cp[3] = std::max(0, thi - tlo + 1);
              for (size_t q = a; q < b; ++q) hs.kslot[r * bh + q] = hsl[q].second;
              for (int32_t t = tlo; t <= thi; ++t, ++nd)
                fill_desc(hs.kdesc.data() + (r * mt_used + nd) * dw, t, pos, j * bh, bh, H, K);
            }
            ++nc;
            a = b;
          }
          if (pass == 0) {
            ncomp[r] = nc;
            nchunk[r] = nk;
          }
        }
    if (pass == 0) {
      hs.max_comp = std::max<int32_t>(1, *std::max_element(ncomp.begin(), ncomp.end()));
      hs.max_chunks = std::max<int32_t>(1, *std::max_element(nchunk.begin(), nchunk.end()));
    }
  }
  hs.mt = mt_used;
  return DODE_OK;
}

dode_status check_params(const dode_spgd_params* p) {
  if (!p) return fail(DODE_ERR_ARG, "params is NULL");
  if (p->epochs < 0) return fail(DODE_ERR_ARG, "epochs=%d is negative", p->epochs);
  if (p->batch_rows < 1) return fail(DODE_ERR_ARG, "batch_rows=%d must be >= 1", p->batch_rows);
  if (!(p->eta > 0) || !std::isfinite(p->eta)) return fail(DODE_ERR_ARG, "eta must be > 0");
  if (!(p->eps >= 0) || !std::isfinite(p->eps)) return fail(DODE_ERR_ARG, "eps must be >= 0");
  if (p->optimizer != 0 && p->optimizer != 1)
    return fail(DODE_ERR_ARG, "optimizer=%d (0 Adagrad, 1 fixed step)", p->optimizer);
  if (p->kernel_path < 0 || p->kernel_path > 3)
    return fail(DODE_ERR_ARG,
                "kernel_path=%d (0 best, 1 sparse, 2 one launch per minibatch, 3 one per epoch)",
                p->kernel_path);
  if (p->day_tile != 0 && p->day_tile != 16 && p->day_tile != 32 && p->day_tile != 64)
    return fail(DODE_ERR_ARG, "day_tile=%d (0 = tune, 16, 32 or 64)", p->day_tile);
  if (p->refine_steps < 0 || p->refine_steps > 16)
    return fail(DODE_ERR_ARG, "refine_steps=%d outside [0, 16]", p->refine_steps);
  if (p->adj_order < 0 || p->adj_order > 2)
    return fail(DODE_ERR_ARG, "adj_order=%d (0, 1 or 2)", p->adj_order);
  if (p->adj_order == 2 && p->day_tile == 64)
    return fail(DODE_ERR_ARG, "adj_order 2 needs day_tile 16 or 32 (or 0 to tune)");
  if (p->slabs < 0 || p->slabs > 64)
    return fail(DODE_ERR_ARG, "slabs=%d outside [0, 64]", p->slabs);
  return DODE_OK;
}

dode_status scan_finite(const dode_dar* dar, const void* X, int64_t n, hipStream_t s) {
  DevBuf flag;
  HIP_TRY(flag.alloc(4, s));
  HIP_TRY(hipMemsetAsync(flag.p, 0, 4, s));
  HIP_TRY(check_finite(dar->storage == DODE_F64, X, n, flag.as<int32_t>(), s));
  int32_t h = 0;
  HIP_TRY(hipMemcpyAsync(&h, flag.p, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (h) return fail(DODE_ERR_NONFINITE, "X holds NaN or Inf");
  return DODE_OK;
}

}  // namespace

bool is_f64(const dode_dar* d) { return d->storage == DODE_F64; }

// ------------------------------------------------------ number formats --
uint16_t host_f64_to_bf16(double v) {
  if (std::isnan(v)) return 0x7FC0;
  const uint16_t sign = std::signbit(v) ? 0x8000 : 0;
  const double a = std::fabs(v);
  if (a == 0.0) return sign;
  if (a < 0x1p-126) {   // bfloat16 subnormals: multiples of 2^-133
    const double m = std::nearbyint(a * 0x1p133);
    return sign | static_cast<uint16_t>(m);
  }
  int e = 0;
  std::frexp(a, &e);                                   // a = f 2^e, f in [0.5, 1)
  double M = std::nearbyint(std::ldexp(a, 8 - e));    // 8 significant bits, ties to even
  if (M >= 256.0) { M = 128.0; ++e; }
  if (e - 1 > 127) return sign | 0x7F80;               // overflow to infinity
  const float f = static_cast<float>(std::ldexp(M, e - 8));
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return sign | static_cast<uint16_t>(u >> 16);
}

double host_bf16_to_f64(uint16_t b) {
  const uint32_t u = static_cast<uint32_t>(b) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

uint8_t host_f64_to_e4m3(double v) {
  const uint8_t sign = std::signbit(v) ? 0x80 : 0;
  const double a = std::fabs(v);
  if (!(a < 448.0)) return sign | 0x7E;   // saturate at the largest finite value
  if (a < 0x1p-6) return sign | static_cast<uint8_t>(std::nearbyint(a * 512.0));
  int e = 0;
  const double f = std::frexp(a, &e);
  int E = e - 1;
  int m = static_cast<int>(std::nearbyint((2.0 * f - 1.0) * 8.0));
  if (m == 8) { m = 0; ++E; }
  int code = ((E + 7) << 3) | m;
  if (code > 0x7E) code = 0x7E;
  return sign | static_cast<uint8_t>(code);
}

double host_e4m3_to_f64(uint8_t b) {
  const int e = (b >> 3) & 0xF, m = b & 7;
  const double v = e == 0 ? m * 0x1p-9 : std::ldexp(1.0 + m / 8.0, e - 7);
  return (b & 0x80) ? -v : v;
}

namespace {

hipEvent_t plan_event(dode_plan* p) {
  if (p->event_next < p->event_pool.size()) return p->event_pool[p->event_next++];
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  p->event_pool.push_back(e);
  p->event_next = p->event_pool.size();
  return e;
}

// Launch `f` and, when timing is on, bracket it with an event pair of kind k.
template <typename F>
hipError_t timed(dode_plan* p, int k, hipStream_t s, F&& f) {
  if (!p->timing) return f();
  hipEvent_t a = plan_event(p), b = plan_event(p);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, s);
  if (e != hipSuccess) return e;
  e = f();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, s);
  p->pending[k].push_back({a, b});
  return e;
}

}  // namespace

namespace {

// Minibatch j of epoch e on the plan's state: forward + residual, then
// adjoint + step + projection.
dode_status run_chunk(dode_plan* plan, const ChunkSched& cs, const CompSched* ks,
                      const ChunkList* ckl, hipStream_t s, bool corr = false, int32_t slab = -1) {
  const dode_dar* dar = plan->dar;
  const Layout& ly = plan->ly;
  if (plan->use_mfma) {
    const DayGroups dg = plan->slab_groups(slab);
    float* R = static_cast<float*>(plan->d_R);
    float* Q = static_cast<float*>(plan->d_Q);
    float* A = static_cast<float*>(plan->d_A);
    const float* X = static_cast<const float*>(plan->d_X);
    if (plan->one_launch && ks && !corr) {
      HIP_TRY(timed(plan, 1, s, [&] { return mfma_minibatch(dar, *ks, dg, ly, X, R, Q, A, plan->sa, s); }));
      return DODE_OK;
    }
    const dode_plan::WaveTables& wt =
        corr ? plan->wt_full : plan->wt_mb[slab < 0 || plan->n_slabs <= 1 ? 0 : slab];
    const int o = cs.order;
    HIP_TRY(timed(plan, 0, s, [&] {
      return mfma_chunk_resid(dar, cs, wt.fwd, wt.n_fwd, plan->day_tile, ly, Q, X, R, corr, s);
    }));
    if (corr && plan->adj_order == 2 && plan->d_kchunk_full) {
      // refinement steps: the chunked adjoint over every departure interval
      const ChunkList full = plan->chunks_full();
      HIP_TRY(timed(plan, 1, s, [&] {
        return mfma_adj_chunks(dar, full, wt.adj[2], wt.n_adj[2], plan->day_tile, ly, R, Q, A,
                               plan->sa, true, s);
      }));
      return DODE_OK;
    }
    if (o == 2 && ckl && !corr) {
      HIP_TRY(timed(plan, 1, s, [&] {
        return mfma_adj_chunks(dar, *ckl, wt.adj[2], wt.n_adj[2], plan->day_tile, ly, R, Q, A,
                               plan->sa, false, s);
      }));
      return DODE_OK;
    }
    HIP_TRY(timed(plan, 1, s, [&] {
      return mfma_chunk_adj_step(dar, cs, wt.adj[o], wt.n_adj[o], plan->day_tile, ly, R, Q, A,
                                 plan->sa, corr, s);
    }));
    return DODE_OK;
  }
  const int32_t* dc = plan->d_dc;
  HIP_TRY(timed(plan, 0, s, [&] {
    return plain_chunk_resid(dar, dc, 0, cs, ly, plan->d_Q, plan->d_X, plan->d_R, plan->D, s);
  }));
  HIP_TRY(timed(plan, 1, s, [&] {
    return plain_chunk_adj_step(dar, dc, 0, cs, ly, plan->d_R, plan->d_Q, plan->d_A, plan->D,
                                plan->sa, s);
  }));
  return DODE_OK;
}

dode_status run_minibatch(dode_plan* plan, int32_t e, int32_t j, hipStream_t s, int32_t slab = -1) {
  const CompSched ks = plan->comps(e, j);
  const ChunkList ckl = plan->chunks(e, j);
  return run_chunk(plan, plan->chunk(e, j), &ks, &ckl, s, false, slab);
}

// The refinement steps that end every epoch: full-batch steps on the
// corrected values (schedule independent of the epoch).
dode_status run_refinement(dode_plan* plan, hipStream_t s) {
  for (int32_t r = 0; r < plan->refine_steps; ++r)
    if (dode_status st = run_chunk(plan, plan->chunk_full(), nullptr, nullptr, s, true)) return st;
  return DODE_OK;
}

// Polls of a persistent launch's grid barrier before it gives up (about a
// second); DODE_PERSIST_SPIN_LIMIT overrides it (tests of the error path).
uint32_t persist_spin_limit() {
  const char* v = getenv("DODE_PERSIST_SPIN_LIMIT");
  return v && *v ? (uint32_t)strtoul(v, nullptr, 10) : (1u << 20);
}

// Every minibatch of epoch e in one cooperative launch (kernel_path 3).
dode_status run_persistent(dode_plan* plan, int32_t e, hipStream_t s) {
  if (!plan->d_mb) {
    std::vector<PersistMinibatch> mb(plan->nch);
    for (int32_t j = 0; j < plan->nch; ++j)
      mb[j] = PersistMinibatch{plan->chunk_dev(j), plan->chunks(-1, j)};
    HIP_TRY(hipMalloc(&plan->d_mb, mb.size() * sizeof(PersistMinibatch)));
    HIP_TRY(hipMemcpy(plan->d_mb, mb.data(), mb.size() * sizeof(PersistMinibatch),
                      hipMemcpyHostToDevice));
    HIP_TRY(hipMalloc(&plan->d_bar, sizeof(PersistBarrier)));
  }
  HIP_TRY(fill_zero(false, plan->d_bar, sizeof(PersistBarrier) / 4, s));
  const dode_plan::WaveTables& wt = plan->wt_mb[0];
  const int o = plan->adj_order;
  HIP_TRY(timed(plan, 1, s, [&] {
    return mfma_epoch_persistent(plan->dar, plan->d_mb, plan->nch, e, wt.fwd, wt.n_fwd, wt.adj[o],
                                 wt.n_adj[o], o, plan->day_tile, plan->ly,
                                 static_cast<const float*>(plan->d_X), static_cast<float*>(plan->d_R),
                                 static_cast<float*>(plan->d_Q), static_cast<float*>(plan->d_A),
                                 plan->sa, plan->d_bar, persist_spin_limit(), s);
  }));
  return DODE_OK;
}

// Every minibatch of epoch e (e < 0: the epoch in the device counter, for
// graph capture), then the refinement steps.  With day slabs, slab k runs its
// minibatches on its own stream, all slabs at the same time: their days are
// disjoint, and one slab's launches fill the others' ramp and tail.  While
// kernel timing is on the slabs run one after another on `s`, so each event
// pair brackets one launch running alone.
dode_status run_epoch(dode_plan* plan, int32_t e, hipStream_t s) {
  if (plan->persistent && e >= 0) {
    if (dode_status st = run_persistent(plan, e, s)) return st;
    return run_refinement(plan, s);
  }
  const int32_t ns = plan->use_mfma ? plan->n_slabs : 1;
  const bool fork = ns > 1 && !plan->timing;
  if (fork) {
    // side stream k-1 runs slab k; the days of different slabs are disjoint
    // (set_slabs made the streams and events, outside any graph capture)
    if ((int32_t)plan->side_streams.size() < ns - 1 || (int32_t)plan->slab_events.size() < ns)
      return fail(DODE_ERR_HIP, "day slab streams missing");
    HIP_TRY(hipEventRecord(plan->slab_events[0], s));
    for (int32_t k = 1; k < ns; ++k)
      HIP_TRY(hipStreamWaitEvent(plan->side_streams[k - 1], plan->slab_events[0], 0));
  }
  for (int32_t k = 0; k < ns; ++k) {
    hipStream_t sk = fork && k > 0 ? plan->side_streams[k - 1] : s;
    for (int32_t j = 0; j < plan->nch; ++j) {
      const CompSched ks = plan->comps(e, j);
      const ChunkList ckl = plan->chunks(e, j);
      const ChunkSched cs = e < 0 ? plan->chunk_dev(j) : plan->chunk(e, j);
      if (dode_status st = run_chunk(plan, cs, &ks, &ckl, sk, false, ns > 1 ? k : -1)) return st;
    }
  }
  if (fork)
    for (int32_t k = 1; k < ns; ++k) {
      HIP_TRY(hipEventRecord(plan->slab_events[k], plan->side_streams[k - 1]));
      HIP_TRY(hipStreamWaitEvent(s, plan->slab_events[k], 0));
    }
  return run_refinement(plan, s);
}

// Capture one epoch (every minibatch, then the epoch-counter increment) into a
// graph on the plan's own stream; replays read the epoch from d_epoch.
dode_status build_epoch_graph(dode_plan* plan) {
  if (plan->graph_exec) return DODE_OK;
  if (!plan->capture_stream)
    HIP_TRY(hipStreamCreateWithFlags(&plan->capture_stream, hipStreamNonBlocking));
  hipStream_t cs = plan->capture_stream;
  HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  dode_status st = run_epoch(plan, -1, cs);
  hipError_t e = st == DODE_OK ? bump_counter(plan->d_epoch, cs) : hipSuccess;
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(cs, &g);
  if (st != DODE_OK || e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    if (st != DODE_OK) return st;
    return fail(DODE_ERR_HIP, "epoch graph capture: %s",
                hipGetErrorString(e != hipSuccess ? e : e2));
  }
  plan->graph = g;
  HIP_TRY(hipGraphInstantiate(&plan->graph_exec, g, nullptr, nullptr, 0));
  return DODE_OK;
}

void drop_epoch_graph(dode_plan* plan) {
  if (plan->graph_exec) (void)hipGraphExecDestroy(plan->graph_exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  plan->graph_exec = nullptr;
  plan->graph = nullptr;
}

void free_tables(dode_plan::WaveTables& t) {
  for (WaveWork* p : {t.fwd, t.adj[0], t.adj[1], t.adj[2]})
    if (p) (void)hipFree(p);
  t = dode_plan::WaveTables{};
}

void free_wave_tables(dode_plan* plan) {
  for (auto& t : plan->wt_mb) free_tables(t);
  plan->wt_mb.clear();
  free_tables(plan->wt_full);
}

hipError_t upload_table(const std::vector<WaveWork>& v, WaveWork** dst, int64_t* n) {
  *n = (int64_t)v.size();
  hipError_t e = hipMalloc(dst, std::max<size_t>(16, v.size() * sizeof(WaveWork)));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, v.data(), v.size() * sizeof(WaveWork), hipMemcpyHostToDevice);
}

// Work tables of every grouped matrix-core launch the plan makes: per slab
// the minibatch forward and both adjoint orders, and on all groups the
// refinement steps' forward and adjoint (every interval a row).
dode_status build_wave_tables(dode_plan* plan, const std::vector<std::vector<int32_t>>& slab_gc,
                              const std::vector<std::vector<int32_t>>& slab_gf,
                              const std::vector<std::vector<int32_t>>& slab_gn) {
  free_wave_tables(plan);
  const dode_dar* dar = plan->dar;
  if (!dar->has_tiles) return DODE_OK;
  for (size_t k = 0; k < slab_gc.size(); ++k) {
    dode_plan::WaveTables t;
    // the chunked adjoint by chunk, then OD tile, with the day groups fastest
    // (measured fastest: neighbouring waves share the up to kChunkT
    // intervals' tiles, and the OD tiles of a chunk its residual rows)
    const auto f = work_table(dar, slab_gc[k], slab_gf[k], slab_gn[k], true, plan->bh, false, false);
    const auto a0 = work_table(dar, slab_gc[k], slab_gf[k], slab_gn[k], false, plan->mt, false, false);
    const auto a1 = work_table(dar, slab_gc[k], slab_gf[k], slab_gn[k], false, plan->kmt, true, false);
    const auto a2 = work_table(dar, slab_gc[k], slab_gf[k], slab_gn[k], false, plan->max_chunks,
                               false, true);
    hipError_t e = upload_table(f, &t.fwd, &t.n_fwd);
    if (e == hipSuccess) e = upload_table(a0, &t.adj[0], &t.n_adj[0]);
    if (e == hipSuccess) e = upload_table(a1, &t.adj[1], &t.n_adj[1]);
    if (e == hipSuccess) e = upload_table(a2, &t.adj[2], &t.n_adj[2]);
    plan->wt_mb.push_back(t);
    HIP_TRY(e);
  }
  if (plan->refine_steps > 0) {
    const int32_t H = dar->dims.H, T = dar->dims.T;
    // full-batch steps: the day groups fastest, so the groups of a cluster
    // read each tile while it is in L2 (the tiles of every interval do not fit)
    const auto f = work_table(dar, plan->h_gc, plan->h_gf, plan->h_gn, true, H, false, true);
    const auto a = work_table(dar, plan->h_gc, plan->h_gf, plan->h_gn, false, T, false, true);
    const auto a2 = work_table(dar, plan->h_gc, plan->h_gf, plan->h_gn, false,
                               std::max<int32_t>(1, plan->full_chunks), false, true);
    HIP_TRY(upload_table(f, &plan->wt_full.fwd, &plan->wt_full.n_fwd));
    HIP_TRY(upload_table(a, &plan->wt_full.adj[0], &plan->wt_full.n_adj[0]));
    HIP_TRY(upload_table(a2, &plan->wt_full.adj[2], &plan->wt_full.n_adj[2]));
  }
  return DODE_OK;
}

// Split the day groups, in order, into n contiguous slabs of about D/n days
// each (a cluster may be split), each slab with its own group list.  Drops a
// captured epoch graph.
dode_status set_slabs(dode_plan* plan, int32_t n) {
  const int32_t G = (int32_t)plan->h_gc.size();
  n = std::max<int32_t>(1, std::min<int32_t>(n, G));
  drop_epoch_graph(plan);
  // the streams and events of concurrent slabs (run_epoch forks and joins them)
  while ((int32_t)plan->side_streams.size() < n - 1) {
    hipStream_t t = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&t, hipStreamNonBlocking));
    plan->side_streams.push_back(t);
  }
  while ((int32_t)plan->slab_events.size() < n) {
    hipEvent_t ev = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    plan->slab_events.push_back(ev);
  }
  if (plan->d_slabs) HIP_TRY(hipFree(plan->d_slabs));
  plan->d_slabs = nullptr;
  plan->slab_off.clear();
  plan->slab_n.clear();
  plan->n_slabs = n;
  if (n == 1) return build_wave_tables(plan, {plan->h_gc}, {plan->h_gf}, {plan->h_gn});
  std::vector<std::vector<int32_t>> sgc, sgf, sgn;
  std::vector<int32_t> buf;
  int64_t days = 0;
  int32_t g = 0;
  for (int32_t k = 0; k < n; ++k) {
    // groups up to the (k+1)-th share of the days; every slab gets at least
    // one group, the last slab all that remain
    const int64_t target = (int64_t)plan->D * (k + 1) / n;
    const int32_t a = g;
    while (g < G) {
      const bool take = k == n - 1 || g == a ||
                        (days + plan->h_gn[g] <= target && G - (g + 1) >= n - k - 1);
      if (!take) break;
      days += plan->h_gn[g];
      ++g;
    }
    const int32_t m = g - a;
    std::vector<int32_t> cl(m), fi(m), co(m), cb(m), cg(m);
    for (int32_t i = 0; i < m; ++i) {
      cl[i] = plan->h_gc[a + i];
      fi[i] = plan->h_gf[a + i];
      co[i] = plan->h_gn[a + i];
    }
    // cluster runs inside the slab: first group and group count of each run
    for (int32_t r0 = 0; r0 < m;) {
      int32_t r1 = r0 + 1;
      while (r1 < m && cl[r1] == cl[r0]) ++r1;
      for (int32_t i = r0; i < r1; ++i) {
        cb[i] = r0;
        cg[i] = r1 - r0;
      }
      r0 = r1;
    }
    plan->slab_off.push_back((int64_t)buf.size());
    plan->slab_n.push_back(m);
    for (const auto* v : {&cl, &fi, &co, &cb, &cg}) buf.insert(buf.end(), v->begin(), v->end());
    sgc.push_back(cl);
    sgf.push_back(fi);
    sgn.push_back(co);
  }
  HIP_TRY(hipMalloc(&plan->d_slabs, std::max<size_t>(buf.size() * 4, 16)));
  HIP_TRY(hipMemcpy(plan->d_slabs, buf.data(), buf.size() * 4, hipMemcpyHostToDevice));
  return build_wave_tables(plan, sgc, sgf, sgn);
}

// Day groups of `tile` days: each cluster's plan days, in order, cut into
// groups of at most `tile`.  Replaces the device list and drops a captured
// epoch graph (it holds the old list).
dode_status set_day_groups(dode_plan* plan, int32_t tile) {
  std::vector<int32_t> gc, gf, gn, gb, gk;
  int32_t start = 0;
  for (int32_t c = 0; c < plan->C; ++c) {
    const int32_t n = plan->cluster_days[c];
    const int32_t base = (int32_t)gc.size(), ng = (n + tile - 1) / tile;
    for (int32_t f = 0; f < n; f += tile) {
      gc.push_back(c);
      gf.push_back(start + f);
      gn.push_back(std::min<int32_t>(tile, n - f));
      gb.push_back(base);
      gk.push_back(ng);
    }
    start += n;
  }
  std::vector<int32_t> buf;
  for (const auto* v : {&gc, &gf, &gn, &gb, &gk}) buf.insert(buf.end(), v->begin(), v->end());
  drop_epoch_graph(plan);
  if (plan->d_groups) HIP_TRY(hipFree(plan->d_groups));
  plan->d_groups = nullptr;
  HIP_TRY(hipMalloc(&plan->d_groups, std::max<size_t>(buf.size() * 4, 16)));
  HIP_TRY(hipMemcpy(plan->d_groups, buf.data(), buf.size() * 4, hipMemcpyHostToDevice));
  plan->n_groups = (int32_t)gc.size();
  plan->day_tile = tile;
  plan->h_gc = gc;
  plan->h_gf = gf;
  plan->h_gn = gn;
  return set_slabs(plan, plan->n_slabs);
}

// Matrix-core schedule choices made in this process, keyed by what decides
// the fastest candidate: shapes, minibatch, storage, cluster sizes and GPU.
std::mutex g_tune_mu;
struct TunedSchedule {
  int32_t day_tile, adj_order, n_slabs;
};
std::map<std::string, TunedSchedule> g_tuned;

std::string tune_key(const dode_plan* plan) {
  const dode_dims& dm = plan->dar->dims;
  hipDeviceProp_t prop{};
  std::string arch = hipGetDeviceProperties(&prop, plan->device) == hipSuccess ? prop.gcnArchName : "?";
  std::string k = arch + "|" + std::to_string(dm.P) + "," + std::to_string(dm.L) + "," +
                  std::to_string(dm.T) + "," + std::to_string(dm.H) + "," + std::to_string(dm.K) +
                  "|" + std::to_string(plan->bh) + "|" + std::to_string((int)plan->dar->storage) +
                  "|" + std::to_string(plan->refine_steps) + "|";
  for (int32_t n : plan->cluster_days) k += std::to_string(n) + ",";
  return k;
}

// Schedule file named by DODE_SCHEDULE_CACHE (none when unset): one line per
// choice, "<key>\t<day tile> <adjoint order> <slabs> <ms>".  Entries that do
// not parse or name no valid schedule are skipped; the last valid entry of a
// key wins.
bool valid_schedule(const TunedSchedule& t) {
  return (t.day_tile == 16 || t.day_tile == 32 || t.day_tile == 64) && t.adj_order >= 0 &&
         t.adj_order <= 2 && !(t.adj_order == 2 && t.day_tile == 64) && t.n_slabs >= 1 &&
         t.n_slabs <= 64;
}

bool read_schedule_file(const std::string& key, TunedSchedule* out) {
  const char* path = getenv("DODE_SCHEDULE_CACHE");
  if (!path || !*path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  bool found = false;
  char line[1024];
  while (fgets(line, sizeof line, f)) {
    char* tab = strchr(line, '\t');
    if (!tab || std::string(line, tab - line) != key) continue;
    TunedSchedule t{};
    if (sscanf(tab + 1, "%d %d %d", &t.day_tile, &t.adj_order, &t.n_slabs) == 3 &&
        valid_schedule(t)) {
      *out = t;
      found = true;
    }
  }
  fclose(f);
  return found;
}

void append_schedule_file(const std::string& key, const TunedSchedule& t, double ms) {
  const char* path = getenv("DODE_SCHEDULE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;   // the choice still holds for this process
  fprintf(f, "%s\t%d %d %d %.6f\n", key.c_str(), t.day_tile, t.adj_order, t.n_slabs, ms);
  fclose(f);
}

// Choose the matrix-core schedule on the loaded state: every day tile
// (16, 32, 64) with the three adjoint item orders (no chunked adjoint with
// 64-day waves) and 1, 2 or 4 day slabs, each timed over one whole epoch
// (epoch 0) after one warm-up minibatch, fastest kept and remembered for the
// same key in this process and in the schedule file.  The runs change the plan's Q and A:
// the caller reloads them.
dode_status tune_schedule(dode_plan* plan, hipStream_t s) {
  static const int32_t kTiles[] = {16, 32, 64};
  static const int32_t kSlabs[] = {1, 2, 4};
  const std::string key = tune_key(plan);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tuned.find(key);
    TunedSchedule known{};
    if (it != g_tuned.end() || read_schedule_file(key, &known)) {
      if (it != g_tuned.end()) known = it->second;
      g_tuned[key] = known;
      plan->adj_order = known.adj_order;
      plan->n_slabs = known.n_slabs;
      plan->n_timed = 0;
      plan->tune_ms = 0.0;
      return set_day_groups(plan, known.day_tile);
    }
  }
  const bool timing = plan->timing;
  plan->timing = false;
  hipEvent_t ev[2] = {nullptr, nullptr};
  dode_status st = DODE_OK;
  float best_ms = 0.f;
  TunedSchedule best{32, 1, 1};
  int32_t n = 0;
  for (int k = 0; k < 2 && st == DODE_OK; ++k)
    if (hipEventCreate(&ev[k]) != hipSuccess) st = fail(DODE_ERR_HIP, "hipEventCreate failed");
  for (int32_t tile : kTiles)
    for (int32_t order = 0; order < 3; ++order)
      for (int32_t slabs : kSlabs) {
        if (st != DODE_OK) break;
        if (order == 2 && tile == 64) continue;   // the chunked adjoint has no 64-day waves
        plan->n_slabs = slabs;
        if ((st = set_day_groups(plan, tile)) != DODE_OK) break;
        if (slabs > 1 && plan->n_slabs != slabs) continue;   // fewer groups than slabs
        plan->adj_order = order;
        if ((st = run_minibatch(plan, 0, 0, s)) != DODE_OK) break;
        hipError_t e = hipEventRecord(ev[0], s);
        if (e == hipSuccess) st = run_epoch(plan, 0, s);
        if (st != DODE_OK) break;
        if (e == hipSuccess) e = hipEventRecord(ev[1], s);
        if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
        if (e != hipSuccess) {
          st = fail(DODE_ERR_HIP, "schedule tuning: %s", hipGetErrorString(e));
          break;
        }
        if (n++ == 0 || ms < best_ms) {
          best_ms = ms;
          best = TunedSchedule{tile, order, slabs};
        }
      }
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  plan->timing = timing;
  if (st != DODE_OK) return st;
  plan->adj_order = best.adj_order;
  plan->n_slabs = best.n_slabs;
  plan->n_timed = n;
  plan->tune_ms = best_ms;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tuned[key] = best;
    append_schedule_file(key, best, best_ms);
  }
  return set_day_groups(plan, best.day_tile);
}

}  // namespace

// ---------------------------------------- scratch of dode_loss_noalloc --
// The per-row loss partials of dode_loss_noalloc live in this fixed device
// array instead of a per-call allocation.  Each GPU that runs the call holds
// its own copy until the process ends; host code reaches it only through the
// per-device address taken once with hipGetSymbolAddress.
constexpr size_t kLossScratchBytes = size_t(4) << 20;   // 4 MiB per device
static __device__ __align__(256) double scratch[kLossScratchBytes / sizeof(double)];

namespace {

std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;   // device address of `scratch`, per device

// Address of the current device's `scratch`, looked up on the first call on
// that device.
dode_status loss_scratch(int dev, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(DODE_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return DODE_OK;
}

}  // namespace

// ================================================================== ABI ==
extern "C" {

const char* dode_last_error(void) { return g_err.c_str(); }

void dode_spgd_defaults(dode_spgd_params* p) {
  if (!p) return;
  p->epochs = 300;
  p->batch_rows = 8192;
  p->eta = 5.0;
  p->eps = 1e-10;
  p->optimizer = 0;
  p->check_finite = 1;
  p->kernel_path = 0;
  p->use_graph = 1;
  p->day_tile = 32;
  p->refine_steps = 0;
  p->adj_order = 1;
  p->slabs = 1;
}

namespace {

// Sliced layout of n lines whose entries are ptr[i] .. ptr[i+1]-1: slice g
// holds lines 64g .. 64g+63.  With `ranked`, the lines of a slice take its
// lanes in order of decreasing degree (ties by index), else line i takes lane
// i%64.  Unpaired, entry k of the line in lane r sits at off + 64k + r; paired,
// entries come two by two, entry k at off + 128(k/2) + 2r + k%2, so a lane
// reads two neighbouring entries with one load.  A slice is as long as its
// longest line (rounded up to even when paired).  Returns the slots per block.
int64_t build_slices(int32_t n, const std::vector<int32_t>& ptr, bool ranked, bool paired,
                     std::vector<int32_t>& off, std::vector<int32_t>& first,
                     std::vector<int32_t>& pos) {
  const int32_t ng = (n + 63) / 64;
  off.assign(ng, 0);
  first.assign(n, 0);
  pos.assign(ptr[n], 0);
  int64_t len = 0;
  std::vector<int32_t> lines;
  for (int32_t g = 0; g < ng; ++g) {
    lines.clear();
    int32_t width = 0;
    for (int32_t i = 64 * g; i < std::min(n, 64 * g + 64); ++i) {
      lines.push_back(i);
      width = std::max(width, ptr[i + 1] - ptr[i]);
    }
    if (ranked)
      std::stable_sort(lines.begin(), lines.end(), [&](int32_t x, int32_t y) {
        return ptr[x + 1] - ptr[x] > ptr[y + 1] - ptr[y];
      });
    off[g] = (int32_t)len;
    for (size_t lane = 0; lane < lines.size(); ++lane)
      first[lines[lane]] = (int32_t)(len + (paired ? 2 : 1) * lane);
    len += 64 * (int64_t)(paired ? (width + 1) / 2 * 2 : width);
  }
  for (int32_t i = 0; i < n; ++i)
    for (int32_t k = 0; k < ptr[i + 1] - ptr[i]; ++k)
      pos[ptr[i] + k] = paired ? first[i] + 128 * (k >> 1) + (k & 1) : first[i] + 64 * k;
  return len;
}

}  // namespace

dode_status dar_destroy(dode_dar* dar) {
  if (!dar) return DODE_OK;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(dar->device);
  for (void* p : {(void*)dar->d_row_ptr, (void*)dar->d_col, (void*)dar->d_col_ptr,
                  (void*)dar->d_row, (void*)dar->d_csc2csr, dar->d_W, dar->d_WT,
                  (void*)dar->d_scale, (void*)dar->d_tile_meta, dar->d_Fv, dar->d_Gv,
                  dar->d_Fc, dar->d_Gc,
                  (void*)dar->d_row_of_nz, (void*)dar->d_sr_first, (void*)dar->d_sr_col,
                  (void*)dar->d_sr_pos, (void*)dar->d_sc_off, (void*)dar->d_sc_row,
                  (void*)dar->d_sc_pos, (void*)dar->d_posf, (void*)dar->d_posg})
    if (p) (void)hipFree(p);
  (void)hipSetDevice(cur);
  delete dar;
  return DODE_OK;
}

dode_status dar_create(const dode_dims* dims, int32_t n_clusters, const int32_t* row_ptr,
                       const int32_t* col_idx, const double* const* values, dode_dtype storage,
                       void* stream, dode_dar** out) {
  return dar_create_ex(dims, n_clusters, row_ptr, col_idx, values, storage, 0, stream, out);
}

dode_status dar_create_ex(const dode_dims* dims, int32_t n_clusters, const int32_t* row_ptr,
                          const int32_t* col_idx, const double* const* values,
                          dode_dtype storage, int32_t flags, void* stream, dode_dar** out) {
  if (!out) return fail(DODE_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (flags & ~DODE_DAR_CORRECTION) return fail(DODE_ERR_ARG, "unknown flags 0x%x", flags);
  if ((flags & DODE_DAR_CORRECTION) && storage != DODE_FP8_E4M3)
    return fail(DODE_ERR_ARG, "DODE_DAR_CORRECTION applies to FP8 storage only");
  if (dode_status st = check_dims(dims)) return st;
  if (n_clusters < 1) return fail(DODE_ERR_ARG, "n_clusters=%d must be >= 1", n_clusters);
  if (!row_ptr || !col_idx || !values) return fail(DODE_ERR_ARG, "pattern or values is NULL");
  if (storage < DODE_F64 || storage > DODE_FP8_E4M3)
    return fail(DODE_ERR_DTYPE, "unknown storage type %d", (int)storage);
  const dode_dims dm = *dims;
  if (row_ptr[0] != 0) return fail(DODE_ERR_SHAPE, "row_ptr[0] must be 0");
  for (int32_t a = 0; a < dm.L; ++a) {
    if (row_ptr[a + 1] < row_ptr[a]) return fail(DODE_ERR_SHAPE, "row_ptr decreases at %d", a);
    for (int32_t j = row_ptr[a]; j < row_ptr[a + 1]; ++j) {
      if (col_idx[j] < 0 || col_idx[j] >= dm.P)
        return fail(DODE_ERR_SHAPE, "col_idx[%d]=%d outside [0, P)", j, col_idx[j]);
      if (j > row_ptr[a] && col_idx[j] <= col_idx[j - 1])
        return fail(DODE_ERR_SHAPE, "col_idx not strictly increasing in row %d", a);
    }
  }
  const int64_t nnz = row_ptr[dm.L];
  for (int32_t c = 0; c < n_clusters; ++c)
    if (!values[c]) return fail(DODE_ERR_ARG, "values[%d] is NULL", c);
  const int64_t cstride = (int64_t)dm.K * dm.T * nnz;
  for (int32_t c = 0; c < n_clusters; ++c) {
    std::vector<char> bad(dm.K, 0);
    host_parallel_for(dm.K, [&](int64_t l0, int64_t l1) {
      for (int64_t l = l0; l < l1; ++l)
        for (int32_t t = 0; t < std::min<int32_t>(dm.T, dm.H - (int32_t)l); ++t)
          for (int64_t j = 0; j < nnz; ++j)
            if (!std::isfinite(values[c][((int64_t)l * dm.T + t) * nnz + j])) bad[l] = 1;
    });
    for (char b : bad)
      if (b) return fail(DODE_ERR_NONFINITE, "values[%d] holds NaN or Inf", c);
  }

  // every early return frees what was allocated so far
  std::unique_ptr<dode_dar, dode_status (*)(dode_dar*)> d(new dode_dar(), dar_destroy);
  d->dims = dm;
  d->C = n_clusters;
  d->nnz = nnz;
  d->storage = storage;
  d->has_corr = (flags & DODE_DAR_CORRECTION) != 0;
  HIP_TRY(hipGetDevice(&d->device));
  d->h_row_ptr.assign(row_ptr, row_ptr + dm.L + 1);
  d->h_col.assign(col_idx, col_idx + nnz);
  // CSC by OD, with the map back to CSR slots
  d->h_col_ptr.assign(dm.P + 1, 0);
  for (int64_t j = 0; j < nnz; ++j) d->h_col_ptr[col_idx[j] + 1]++;
  for (int32_t p = 0; p < dm.P; ++p) d->h_col_ptr[p + 1] += d->h_col_ptr[p];
  d->h_row.resize(nnz);
  d->h_csc2csr.resize(nnz);
  {
    std::vector<int32_t> fillp(d->h_col_ptr.begin(), d->h_col_ptr.end() - 1);
    for (int32_t a = 0; a < dm.L; ++a)
      for (int32_t j = row_ptr[a]; j < row_ptr[a + 1]; ++j) {
        const int32_t jj = fillp[col_idx[j]]++;
        d->h_row[jj] = a;
        d->h_csc2csr[jj] = j;
      }
  }
  hipStream_t s = as_stream(stream);
  auto dev_copy = [&](int32_t** dst, const std::vector<int32_t>& src) -> hipError_t {
    hipError_t e = hipMalloc(dst, std::max<size_t>(16, src.size() * 4));
    if (e != hipSuccess) return e;
    d->device_bytes += src.size() * 4;
    return hipMemcpy(*dst, src.data(), src.size() * 4, hipMemcpyHostToDevice);
  };
  HIP_TRY(dev_copy(&d->d_row_ptr, d->h_row_ptr));
  HIP_TRY(dev_copy(&d->d_col, d->h_col));
  HIP_TRY(dev_copy(&d->d_col_ptr, d->h_col_ptr));
  HIP_TRY(dev_copy(&d->d_row, d->h_row));
  HIP_TRY(dev_copy(&d->d_csc2csr, d->h_csc2csr));
  {
    std::vector<int32_t> rows(nnz);
    for (int32_t a = 0; a < dm.L; ++a)
      for (int32_t j = row_ptr[a]; j < row_ptr[a + 1]; ++j) rows[j] = a;
    HIP_TRY(dev_copy(&d->d_row_of_nz, rows));
  }
  // sliced value layouts: W by link (ranked by degree, entries in pairs), WT
  // by OD; each line's entries keep their CSR / CSC order
  std::vector<int32_t> sr_off, sr_first, sr_pos, sc_off, sc_first, sc_pos;
  d->sr_len = build_slices(dm.L, d->h_row_ptr, true, true, sr_off, sr_first, sr_pos);
  d->sc_len = build_slices(dm.P, d->h_col_ptr, false, false, sc_off, sc_first, sc_pos);
  if (d->sr_len > INT32_MAX || d->sc_len > INT32_MAX) {
    dar_destroy(d.release());
    return fail(DODE_ERR_SHAPE, "pattern too large for the sliced layout");
  }
  {
    std::vector<int32_t> sr_col(d->sr_len, 0), sc_row(d->sc_len, 0);
    for (int64_t j = 0; j < nnz; ++j) sr_col[sr_pos[j]] = col_idx[j];
    for (int64_t jj = 0; jj < nnz; ++jj) sc_row[sc_pos[jj]] = d->h_row[jj];
    HIP_TRY(dev_copy(&d->d_sr_first, sr_first));
    HIP_TRY(dev_copy(&d->d_sr_col, sr_col));
    HIP_TRY(dev_copy(&d->d_sr_pos, sr_pos));
    HIP_TRY(dev_copy(&d->d_sc_off, sc_off));
    HIP_TRY(dev_copy(&d->d_sc_row, sc_row));
    HIP_TRY(dev_copy(&d->d_sc_pos, sc_pos));
  }

  const size_t esz = storage == DODE_F64 ? 8 : storage == DODE_F32 ? 4 : storage == DODE_BF16 ? 2 : 1;
  const int64_t cstride_r = (int64_t)dm.K * dm.T * d->sr_len, cstride_c = (int64_t)dm.K * dm.T * d->sc_len;
  const size_t vbytes_r = (size_t)n_clusters * cstride_r * esz, vbytes_c = (size_t)n_clusters * cstride_c * esz;
  HIP_TRY(hipMalloc(&d->d_W, std::max<size_t>(16, vbytes_r)));
  HIP_TRY(hipMalloc(&d->d_WT, std::max<size_t>(16, vbytes_c)));
  d->device_bytes += vbytes_r + vbytes_c;
  const int32_t n_ptile = (dm.P + 63) / 64;
  const size_t sbytes = (size_t)n_clusters * dm.K * dm.T * n_ptile * 4;
  if (storage == DODE_FP8_E4M3) {
    HIP_TRY(hipMalloc(&d->d_scale, sbytes));
    d->device_bytes += sbytes;
  }
  const bool tiled = storage == DODE_BF16 || storage == DODE_FP8_E4M3;
  if (tiled) {
    std::string err;
    if (dode_status st = tiles_prepare(d.get(), err)) {
      dar_destroy(d.release());
      return fail(st, "tile layout: %s", err.c_str());
    }
  }
  // host conversion, one cluster at a time: CSR-order codes (for the tiles)
  // and the two sliced copies (padding slots stay zero)
  std::vector<uint8_t> hw(cstride * esz), hws(cstride_r * esz, 0), hwt(cstride_c * esz, 0);
  std::vector<uint16_t> hcorr(d->has_corr ? cstride : 0);
  std::vector<float> hs(storage == DODE_FP8_E4M3 ? (size_t)dm.K * dm.T * n_ptile : 0);
  for (int32_t c = 0; c < n_clusters; ++c) {
    const double* src = values[c];
    if (storage == DODE_FP8_E4M3) {
      host_parallel_for((int64_t)dm.K * dm.T, [&](int64_t b0, int64_t b1) {
        std::vector<double> tmax(n_ptile);
        for (int64_t lt = b0; lt < b1; ++lt) {
          std::fill(tmax.begin(), tmax.end(), 0.0);
          for (int64_t j = 0; j < nnz; ++j)
            tmax[col_idx[j] >> 6] = std::max(tmax[col_idx[j] >> 6], std::fabs(src[lt * nnz + j]));
          for (int32_t i = 0; i < n_ptile; ++i)
            hs[lt * n_ptile + i] = tmax[i] > 0 ? static_cast<float>(tmax[i] / 448.0) : 1.0f;
        }
      });
    }
    host_parallel_for((int64_t)dm.K * dm.T, [&](int64_t b0, int64_t b1) {
    for (int64_t lt = b0; lt < b1; ++lt)
      for (int64_t jj = 0; jj < nnz; ++jj) {
        const int64_t j = d->h_csc2csr[jj];
        const double v = src[lt * nnz + j];
        const int64_t ij = lt * nnz + j;
        const int64_t sj = lt * d->sr_len + sr_pos[j], sjj = lt * d->sc_len + sc_pos[jj];
        switch (storage) {
          case DODE_F64:
            reinterpret_cast<double*>(hw.data())[ij] = v;
            reinterpret_cast<double*>(hws.data())[sj] = v;
            reinterpret_cast<double*>(hwt.data())[sjj] = v;
            break;
          case DODE_F32:
            reinterpret_cast<float*>(hw.data())[ij] = static_cast<float>(v);
            reinterpret_cast<float*>(hws.data())[sj] = static_cast<float>(v);
            reinterpret_cast<float*>(hwt.data())[sjj] = static_cast<float>(v);
            break;
          case DODE_BF16: {
            const uint16_t b = host_f64_to_bf16(v);
            reinterpret_cast<uint16_t*>(hw.data())[ij] = b;
            reinterpret_cast<uint16_t*>(hws.data())[sj] = b;
            reinterpret_cast<uint16_t*>(hwt.data())[sjj] = b;
            break;
          }
          case DODE_FP8_E4M3: {
            const float sc = hs[lt * n_ptile + (col_idx[j] >> 6)];
            const uint8_t b = host_f64_to_e4m3(v / sc);
            hw[ij] = b;
            hws[sj] = b;
            hwt[sjj] = b;
            if (d->has_corr) {
              // the kernels expand a code to bf16(fp32(scale * e4m3)); the
              // correction is what remains, rounded to bf16
              const float prod = static_cast<float>(host_e4m3_to_f64(b)) * sc;
              const double h = host_bf16_to_f64(host_f64_to_bf16(prod));
              hcorr[ij] = host_f64_to_bf16(v - h);
            }
            break;
          }
        }
      }
    });
    HIP_TRY(hipMemcpy(static_cast<uint8_t*>(d->d_W) + c * cstride_r * esz, hws.data(),
                      cstride_r * esz, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(static_cast<uint8_t*>(d->d_WT) + c * cstride_c * esz, hwt.data(),
                      cstride_c * esz, hipMemcpyHostToDevice));
    if (storage == DODE_FP8_E4M3)
      HIP_TRY(hipMemcpy(d->d_scale + (size_t)c * dm.K * dm.T * n_ptile, hs.data(), hs.size() * 4,
                        hipMemcpyHostToDevice));
    if (tiled) {
      std::string err;
      if (dode_status st = tiles_fill_cluster(d.get(), c, hw.data(), err)) {
        dar_destroy(d.release());
        return fail(st, "tile fill: %s", err.c_str());
      }
      if (d->has_corr)
        if (dode_status st = tiles_fill_correction(d.get(), c, hcorr.data(), err)) {
          dar_destroy(d.release());
          return fail(st, "correction tile fill: %s", err.c_str());
        }
    }
  }
  HIP_TRY(hipStreamSynchronize(s));
  *out = d.release();
  return DODE_OK;
}

dode_status dar_info(const dode_dar* dar, dode_dims* dims, int32_t* n_clusters, int64_t* nnz,
                     dode_dtype* storage, int64_t* device_bytes) {
  if (!dar) return fail(DODE_ERR_ARG, "dar handle is NULL");
  if (dims) *dims = dar->dims;
  if (n_clusters) *n_clusters = dar->C;
  if (nnz) *nnz = dar->nnz;
  if (storage) *storage = dar->storage;
  if (device_bytes) *device_bytes = dar->device_bytes;
  return DODE_OK;
}

dode_status dar_set_values(dode_dar* dar, int32_t cluster, const void* W_dev, void* stream) {
  if (dode_status st = check_dar(dar, cluster)) return st;
  if (!W_dev) return fail(DODE_ERR_ARG, "W_dev is NULL");
  if (dar->has_corr)
    return fail(DODE_ERR_UNSUPPORTED, "dar_set_values on a handle with correction tiles");
  if (dar->storage == DODE_FP8_E4M3 && dar->dims.P > 64 * 64)
    return fail(DODE_ERR_UNSUPPORTED, "device FP8 requantisation supports P <= 4096");
  HIP_TRY(quantize_values(dar, cluster, W_dev, as_stream(stream)));
  if (dar->has_tiles) HIP_TRY(update_tiles(dar, cluster, as_stream(stream)));
  return DODE_OK;
}

dode_status dode_apply(const dode_dar* dar, int32_t cluster, const void* Q, int32_t n_days,
                       void* Xhat, void* stream) {
  if (dode_status st = check_dar(dar, cluster)) return st;
  if (dode_status st = check_days(n_days)) return st;
  if (n_days == 0) return DODE_OK;
  if (!Q || !Xhat) return fail(DODE_ERR_ARG, "Q or Xhat is NULL");
  HIP_TRY(plain_apply_rows(dar, nullptr, cluster, day_major(dar->dims), Q, nullptr, Xhat, nullptr, n_days,
                           as_stream(stream)));
  return DODE_OK;
}

dode_status dode_loss(const dode_dar* dar, int32_t cluster, const void* Q, const void* X,
                      int32_t n_days, double* loss, void* stream) {
  if (dode_status st = check_dar(dar, cluster)) return st;
  if (dode_status st = check_days(n_days)) return st;
  if (n_days == 0) return DODE_OK;
  if (!Q || !X || !loss) return fail(DODE_ERR_ARG, "Q, X or loss is NULL");
  hipStream_t s = as_stream(stream);
  DevBuf part;
  HIP_TRY(part.alloc((size_t)n_days * dar->dims.H * 8, s));
  HIP_TRY(plain_apply_rows(dar, nullptr, cluster, day_major(dar->dims), Q, X, nullptr,
                           part.as<double>(), n_days, s));
  HIP_TRY(sum_partials(part.as<double>(), dar->dims.H, n_days, loss, s));
  return DODE_OK;
}

dode_status dode_loss_noalloc(const dode_dar* dar, int32_t cluster, const void* Q, const void* X,
                              int32_t n_days, double* loss, void* stream) {
  if (dode_status st = check_dar(dar, cluster)) return st;
  if (dode_status st = check_days(n_days)) return st;
  if (n_days == 0) return DODE_OK;
  if (!Q || !X || !loss) return fail(DODE_ERR_ARG, "Q, X or loss is NULL");
  const size_t need = (size_t)n_days * dar->dims.H * sizeof(double);
  if (need > kLossScratchBytes)
    return fail(DODE_ERR_ARG,
                "n_days=%d needs %zu bytes of loss scratch, more than the %zu bytes "
                "dode_loss_noalloc holds (at most %zu days with H=%d)",
                n_days, need, kLossScratchBytes,
                kLossScratchBytes / (sizeof(double) * (size_t)dar->dims.H), dar->dims.H);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != dar->device)
    return fail(DODE_ERR_ARG, "the current device %d is not the dar's device %d", dev, dar->device);
  double* part = nullptr;
  if (dode_status st = loss_scratch(dev, &part)) return st;
  hipStream_t s = as_stream(stream);
  // every partial [d][h] is written before it is read: nothing to clear
  HIP_TRY(plain_apply_rows(dar, nullptr, cluster, day_major(dar->dims), Q, X, nullptr, part,
                           n_days, s));
  HIP_TRY(sum_partials(part, dar->dims.H, n_days, loss, s));
  return DODE_OK;
}

dode_status dode_grad(const dode_dar* dar, int32_t cluster, const void* Q, const void* X,
                      int32_t n_days, void* G, void* stream) {
  if (dode_status st = check_dar(dar, cluster)) return st;
  if (dode_status st = check_days(n_days)) return st;
  if (n_days == 0) return DODE_OK;
  if (!Q || !X || !G) return fail(DODE_ERR_ARG, "Q, X or G is NULL");
  hipStream_t s = as_stream(stream);
  DevBuf R;
  HIP_TRY(R.alloc((size_t)n_days * dar->dims.H * dar->dims.L * state_size(dar), s));
  HIP_TRY(plain_apply_rows(dar, nullptr, cluster, day_major(dar->dims), Q, X, R.p, nullptr, n_days, s));
  HIP_TRY(plain_adjoint_rows(dar, nullptr, cluster, day_major(dar->dims), R.p, G, n_days, s));
  return DODE_OK;
}

dode_status dode_metrics(const dode_dar* dar, int32_t cluster, const void* Q, const void* X,
                         int32_t n_days, double* loss, double* kkt, double* r2, void* stream) {
  if (dode_status st = check_dar(dar, cluster)) return st;
  if (dode_status st = check_days(n_days)) return st;
  if (n_days == 0) return DODE_OK;
  if (!Q || !X) return fail(DODE_ERR_ARG, "Q or X is NULL");
  hipStream_t s = as_stream(stream);
  const dode_dims& dm = dar->dims;
  const int32_t n = n_days;
  DevBuf part, lbuf, sumx, sst, R, G;
  HIP_TRY(part.alloc((size_t)n * std::max(dm.H, dm.T) * 8, s));
  HIP_TRY(lbuf.alloc((size_t)n * 8, s));
  if (kkt) {
    HIP_TRY(R.alloc((size_t)n * dm.H * dm.L * state_size(dar), s));
    HIP_TRY(G.alloc((size_t)n * dm.T * dm.P * state_size(dar), s));
  }
  HIP_TRY(plain_apply_rows(dar, nullptr, cluster, day_major(dm), Q, X, kkt ? R.p : nullptr,
                           part.as<double>(), n, s));
  HIP_TRY(sum_partials(part.as<double>(), dm.H, n, lbuf.as<double>(), s));
  if (loss) HIP_TRY(hipMemcpyAsync(loss, lbuf.p, (size_t)n * 8, hipMemcpyDeviceToDevice, s));
  if (kkt) {
    HIP_TRY(plain_adjoint_rows(dar, nullptr, cluster, day_major(dm), R.p, G.p, n, s));
    HIP_TRY(kkt_partials(is_f64(dar), Q, G.p, dm.T, dm.P, n, part.as<double>(), s));
    HIP_TRY(max_partials(part.as<double>(), dm.T, n, kkt, s));
  }
  if (r2) {
    HIP_TRY(sumx.alloc((size_t)n * 8, s));
    HIP_TRY(sst.alloc((size_t)n * 8, s));
    HIP_TRY(x_moment_partials(is_f64(dar), X, dm.H, dm.L, n, nullptr, part.as<double>(), s));
    HIP_TRY(sum_partials(part.as<double>(), dm.H, n, sumx.as<double>(), s));
    HIP_TRY(x_moment_partials(is_f64(dar), X, dm.H, dm.L, n, sumx.as<double>(), part.as<double>(), s));
    HIP_TRY(sum_partials(part.as<double>(), dm.H, n, sst.as<double>(), s));
    HIP_TRY(r2_finish(lbuf.as<double>(), sst.as<double>(), n, r2, s));
  }
  return DODE_OK;
}

dode_status dode_loss_bwd(const dode_dar* dar, int32_t cluster, const void* Q, const void* X,
                          int32_t n_days, double grad_out, void* dQ, void* dW, void* stream) {
  if (dode_status st = check_dar(dar, cluster)) return st;
  if (dode_status st = check_days(n_days)) return st;
  if (!Q || !X) return fail(DODE_ERR_ARG, "Q or X is NULL");
  if (!std::isfinite(grad_out)) return fail(DODE_ERR_ARG, "grad_out is not finite");
  const dode_dims& dm = dar->dims;
  hipStream_t s = as_stream(stream);
  const bool f64 = is_f64(dar);
  DevBuf R;
  HIP_TRY(R.alloc((size_t)std::max(n_days, 1) * dm.H * dm.L * state_size(dar), s));
  if (n_days > 0)
    HIP_TRY(plain_apply_rows(dar, nullptr, cluster, day_major(dm), Q, X, R.p, nullptr, n_days, s));
  if (dQ && n_days > 0) {
    HIP_TRY(plain_adjoint_rows(dar, nullptr, cluster, day_major(dm), R.p, dQ, n_days, s));
    HIP_TRY(scale_state(f64, dQ, (int64_t)n_days * dm.T * dm.P, 2.0 * grad_out, s));
  }
  if (dW) HIP_TRY(loss_bwd_dW(dar, R.p, Q, n_days, 2.0 * grad_out, dW, s));
  return DODE_OK;
}

dode_status dode_routes_destroy(dode_routes* routes) {
  if (!routes) return DODE_OK;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(routes->device);
  if (routes->d_buf) (void)hipFree(routes->d_buf);
  (void)hipSetDevice(cur);
  delete routes;
  return DODE_OK;
}

dode_status dode_routes_create(const dode_dims* dims, int64_t nnz, int32_t n_paths,
                               const int32_t* path_od, const int32_t* pair_ptr,
                               const int32_t* pair_link, const int32_t* pair_nz, void* stream,
                               dode_routes** out) {
  if (!out) return fail(DODE_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (dode_status st = check_dims(dims)) return st;
  if (n_paths < 1 || nnz < 1) return fail(DODE_ERR_ARG, "need n_paths >= 1 and nnz >= 1");
  if (!path_od || !pair_ptr || !pair_link || !pair_nz) return fail(DODE_ERR_ARG, "NULL route array");
  const dode_dims dm = *dims;
  if (pair_ptr[0] != 0) return fail(DODE_ERR_SHAPE, "pair_ptr[0] must be 0");
  for (int32_t k = 0; k < n_paths; ++k) {
    if (path_od[k] < 0 || path_od[k] >= dm.P) return fail(DODE_ERR_SHAPE, "path_od[%d] out of range", k);
    if (pair_ptr[k + 1] < pair_ptr[k]) return fail(DODE_ERR_SHAPE, "pair_ptr decreases at %d", k);
  }
  const int32_t n_pairs = pair_ptr[n_paths];
  std::vector<int32_t> pair_path(n_pairs);
  for (int32_t k = 0; k < n_paths; ++k)
    for (int32_t m = pair_ptr[k]; m < pair_ptr[k + 1]; ++m) {
      if (pair_link[m] < 0 || pair_link[m] >= dm.L) return fail(DODE_ERR_SHAPE, "pair_link[%d]", m);
      if (pair_nz[m] < 0 || pair_nz[m] >= nnz) return fail(DODE_ERR_SHAPE, "pair_nz[%d]", m);
      pair_path[m] = k;
    }
  std::vector<int32_t> od_ptr(dm.P + 1, 0), od_paths(n_paths), nz_ptr(nnz + 1, 0), nz_pairs(n_pairs);
  for (int32_t k = 0; k < n_paths; ++k) od_ptr[path_od[k] + 1]++;
  for (int32_t p = 0; p < dm.P; ++p) od_ptr[p + 1] += od_ptr[p];
  {
    std::vector<int32_t> f(od_ptr.begin(), od_ptr.end() - 1);
    for (int32_t k = 0; k < n_paths; ++k) od_paths[f[path_od[k]]++] = k;
  }
  for (int32_t m = 0; m < n_pairs; ++m) nz_ptr[pair_nz[m] + 1]++;
  for (int64_t j = 0; j < nnz; ++j) nz_ptr[j + 1] += nz_ptr[j];
  {
    std::vector<int32_t> f(nz_ptr.begin(), nz_ptr.end() - 1);
    for (int32_t m = 0; m < n_pairs; ++m) nz_pairs[f[pair_nz[m]]++] = m;
  }
  std::vector<int32_t> buf;
  std::vector<size_t> off;
  auto put = [&](const int32_t* a, size_t n) {
    off.push_back(buf.size());
    buf.insert(buf.end(), a, a + n);
  };
  put(path_od, n_paths);
  put(pair_ptr, n_paths + 1);
  put(pair_nz, n_pairs);
  put(pair_path.data(), n_pairs);
  put(od_ptr.data(), od_ptr.size());
  put(od_paths.data(), n_paths);
  put(nz_ptr.data(), nz_ptr.size());
  put(nz_pairs.data(), n_pairs);
  std::unique_ptr<dode_routes, dode_status (*)(dode_routes*)> r(new dode_routes(),
                                                                 dode_routes_destroy);
  HIP_TRY(hipGetDevice(&r->device));
  HIP_TRY(hipMalloc(&r->d_buf, buf.size() * 4));
  HIP_TRY(hipMemcpy(r->d_buf, buf.data(), buf.size() * 4, hipMemcpyHostToDevice));
  DevRoutes& v = r->dv;
  v = DevRoutes{dm.P, dm.L, dm.T, dm.H, dm.K, n_paths, nnz, n_pairs,
                r->d_buf + off[0], r->d_buf + off[1], r->d_buf + off[2], r->d_buf + off[3],
                r->d_buf + off[4], r->d_buf + off[5], r->d_buf + off[6], r->d_buf + off[7]};
  (void)stream;
  *out = r.release();
  return DODE_OK;
}

dode_status dar_from_logits(const dode_routes* routes, int32_t f64, const void* Rr, const void* z,
                            void* W, void* stream) {
  if (!routes) return fail(DODE_ERR_ARG, "routes is NULL");
  if (!Rr || !z || !W) return fail(DODE_ERR_ARG, "Rr, z or W is NULL");
  hipStream_t s = as_stream(stream);
  DevBuf pi;
  HIP_TRY(pi.alloc((size_t)routes->dv.n_paths * 8, s));
  HIP_TRY(routes_rho(routes->dv, f64 != 0, Rr, z, W, pi.as<double>(), s));
  return DODE_OK;
}

dode_status dar_logits_bwd(const dode_routes* routes, int32_t f64, const void* Rr, const void* z,
                           const void* dW, void* dz, void* stream) {
  if (!routes) return fail(DODE_ERR_ARG, "routes is NULL");
  if (!Rr || !z || !dW || !dz) return fail(DODE_ERR_ARG, "Rr, z, dW or dz is NULL");
  hipStream_t s = as_stream(stream);
  DevBuf pi, dpi;
  HIP_TRY(pi.alloc((size_t)routes->dv.n_paths * 8, s));
  HIP_TRY(dpi.alloc((size_t)routes->dv.n_paths * 8, s));
  HIP_TRY(routes_logits_bwd(routes->dv, f64 != 0, Rr, z, dW, dz, pi.as<double>(), dpi.as<double>(), s));
  return DODE_OK;
}

namespace {

// The path tables are small: check them on the host (every index a kernel
// will use), then the lengths and speeds on the device.
dode_status check_paths_speeds(int32_t n_paths, const int32_t* path_ptr, const int32_t* path_link,
                               int64_t n_pairs, int32_t L, const void* link_len, const void* speed,
                               int32_t n_days, int32_t H_speed, bool f64, hipStream_t s) {
  std::vector<int32_t> hp(n_paths + 1), hl((size_t)n_pairs);
  HIP_TRY(hipMemcpyAsync(hp.data(), path_ptr, hp.size() * 4, hipMemcpyDeviceToHost, s));
  if (n_pairs) HIP_TRY(hipMemcpyAsync(hl.data(), path_link, hl.size() * 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (hp[0] != 0 || hp[n_paths] != n_pairs)
    return fail(DODE_ERR_SHAPE, "path_ptr must run from 0 to n_pairs=%lld", (long long)n_pairs);
  for (int32_t k = 0; k < n_paths; ++k)
    if (hp[k + 1] < hp[k]) return fail(DODE_ERR_SHAPE, "path_ptr decreases at path %d", k);
  for (int64_t m = 0; m < n_pairs; ++m)
    if (hl[m] < 0 || hl[m] >= L)
      return fail(DODE_ERR_SHAPE, "path_link[%lld]=%d outside [0, L)", (long long)m, hl[m]);
  DevBuf flag;
  HIP_TRY(flag.alloc(4, s));
  HIP_TRY(fill_zero(false, flag.p, 1, s));
  HIP_TRY(dar_check_speeds(f64, link_len, L, flag.as<int32_t>(), s));
  HIP_TRY(dar_check_speeds(f64, speed, (int64_t)n_days * L * H_speed, flag.as<int32_t>(), s));
  int32_t h = 0;
  HIP_TRY(hipMemcpyAsync(&h, flag.p, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (h) return fail(DODE_ERR_ARG, "link lengths and speeds must be positive and finite");
  return DODE_OK;
}

}  // namespace

dode_status dode_dar_patterns_from_speeds(int32_t n_paths, const int32_t* path_ptr,
                                          const int32_t* path_link, int64_t n_pairs, int32_t L,
                                          const void* link_len, const void* speed,
                                          int32_t n_patterns, const int32_t* pattern_ptr,
                                          int32_t H_speed, double dt, int32_t H, int32_t K,
                                          int32_t f64, void* Rr, void* cost, void* stream) {
  if (n_patterns < 1 || !pattern_ptr)
    return fail(DODE_ERR_ARG, "n_patterns=%d must be >= 1 and pattern_ptr non-NULL", n_patterns);
  if (pattern_ptr[0] != 0) return fail(DODE_ERR_SHAPE, "pattern_ptr[0] must be 0");
  for (int32_t q = 0; q < n_patterns; ++q)
    if (pattern_ptr[q + 1] <= pattern_ptr[q])
      return fail(DODE_ERR_SHAPE, "pattern %d has no days (pattern_ptr must increase)", q);
  const int32_t n_days = pattern_ptr[n_patterns];
  if (n_paths < 1 || n_pairs < 0 || L < 1 || H_speed < 1 || H < 1)
    return fail(DODE_ERR_SHAPE, "n_paths=%d n_pairs=%lld L=%d n_days=%d H_speed=%d H=%d", n_paths,
                (long long)n_pairs, L, n_days, H_speed, H);
  if (K < 1 || K > kMaxDarLags) return fail(DODE_ERR_SHAPE, "K=%d outside [1, %d]", K, kMaxDarLags);
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DODE_ERR_ARG, "dt=%g must be positive", dt);
  if (!path_ptr || !path_link || !link_len || !speed || !Rr)
    return fail(DODE_ERR_ARG, "path_ptr, path_link, link_len, speed or Rr is NULL");
  hipStream_t s = as_stream(stream);
  // one check of the path tables and of every day's speeds for the whole job
  if (dode_status st = check_paths_speeds(n_paths, path_ptr, path_link, n_pairs, L, link_len, speed,
                                          n_days, H_speed, f64 != 0, s))
    return st;
  // trajectory scratch (and path exit times) for a chunk of days, at most
  // 4 GiB or DODE_DAR_SCRATCH_BYTES (at least one day), shared by the patterns
  const size_t ss = f64 ? 8 : 4;
  const size_t per_day = ((size_t)n_pairs + (cost ? (size_t)n_paths : 0)) * (H + 1) * ss;
  size_t limit = size_t(1) << 32;
  if (const char* e = std::getenv("DODE_DAR_SCRATCH_BYTES")) {
    char* end = nullptr;
    const unsigned long long v = std::strtoull(e, &end, 10);
    if (e[0] < '0' || e[0] > '9' || *end != '\0' || v == 0)
      return fail(DODE_ERR_ARG, "DODE_DAR_SCRATCH_BYTES='%s' is not a positive byte count", e);
    limit = (size_t)v;
  }
  int32_t most = 0;
  for (int32_t q = 0; q < n_patterns; ++q) most = std::max(most, pattern_ptr[q + 1] - pattern_ptr[q]);
  const size_t cap = std::max<size_t>(1, limit / std::max<size_t>(per_day, 1));
  const int32_t chunk = (int32_t)std::min<size_t>((size_t)most, cap);
  DevBuf traj, sums;
  HIP_TRY(traj.alloc(std::max<size_t>(per_day * chunk, 16), s));
  void* exit_time = static_cast<uint8_t*>(traj.p) + (size_t)n_pairs * (H + 1) * ss * chunk;
  if (cost) HIP_TRY(sums.alloc((size_t)n_paths * H * 8, s));
  for (int32_t q = 0; q < n_patterns; ++q) {
    const int32_t d0 = pattern_ptr[q], nd = pattern_ptr[q + 1] - d0;
    const void* sp = static_cast<const uint8_t*>(speed) + (size_t)d0 * L * H_speed * ss;
    void* rq = static_cast<uint8_t*>(Rr) + (size_t)q * K * H * n_pairs * ss;
    void* cq = cost ? static_cast<uint8_t*>(cost) + (size_t)q * H * n_paths * ss : nullptr;
    HIP_TRY(dar_from_speeds(f64 != 0, n_paths, path_ptr, path_link, n_pairs, L, link_len, sp, nd,
                            H_speed, dt, H, K, traj.p, std::min(chunk, nd), rq, exit_time,
                            sums.as<double>(), cq, s));
  }
  return DODE_OK;
}

dode_status dode_dar_costs_from_speeds(int32_t n_paths, const int32_t* path_ptr,
                                       const int32_t* path_link, int64_t n_pairs, int32_t L,
                                       const void* link_len, const void* speed, int32_t n_days,
                                       int32_t H_speed, double dt, int32_t H, int32_t K,
                                       int32_t f64, void* Rr, void* cost, void* stream) {
  if (n_days < 1) return fail(DODE_ERR_SHAPE, "n_days=%d must be >= 1", n_days);
  const int32_t days[2] = {0, n_days};
  return dode_dar_patterns_from_speeds(n_paths, path_ptr, path_link, n_pairs, L, link_len, speed,
                                       1, days, H_speed, dt, H, K, f64, Rr, cost, stream);
}

dode_status dode_dar_from_speeds(int32_t n_paths, const int32_t* path_ptr,
                                 const int32_t* path_link, int64_t n_pairs, int32_t L,
                                 const void* link_len, const void* speed, int32_t n_days,
                                 int32_t H_speed, double dt, int32_t H, int32_t K, int32_t f64,
                                 void* Rr, void* stream) {
  return dode_dar_costs_from_speeds(n_paths, path_ptr, path_link, n_pairs, L, link_len, speed,
                                    n_days, H_speed, dt, H, K, f64, Rr, nullptr, stream);
}

dode_status dode_path_costs(int32_t n_paths, const int32_t* path_ptr, const int32_t* path_link,
                            int64_t n_pairs, int32_t L, const void* link_len, const void* speed,
                            int32_t n_days, int32_t H_speed, double dt, int32_t T, int32_t f64,
                            void* cost, void* stream) {
  if (n_paths < 1 || n_pairs < 0 || L < 1 || n_days < 1 || H_speed < 1 || T < 1)
    return fail(DODE_ERR_SHAPE, "n_paths=%d n_pairs=%lld L=%d n_days=%d H_speed=%d T=%d", n_paths,
                (long long)n_pairs, L, n_days, H_speed, T);
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DODE_ERR_ARG, "dt=%g must be positive", dt);
  if (!path_ptr || !path_link || !link_len || !speed || !cost)
    return fail(DODE_ERR_ARG, "path_ptr, path_link, link_len, speed or cost is NULL");
  if ((int64_t)n_paths * T > (int64_t(1) << 31))
    return fail(DODE_ERR_SHAPE, "n_paths * T too large");
  hipStream_t s = as_stream(stream);
  if (dode_status st = check_paths_speeds(n_paths, path_ptr, path_link, n_pairs, L, link_len, speed,
                                          n_days, H_speed, f64 != 0, s))
    return st;
  // FP64 slice sums: slices of 4 days (more when the scratch would pass 256 MiB)
  const size_t per_slice_bytes = (size_t)n_paths * T * 8;
  const size_t cap_slices = std::max<size_t>(1, (size_t(256) << 20) / per_slice_bytes);
  const size_t groups = ((size_t)n_days + 3) / 4;
  const int32_t per_slice = 4 * (int32_t)((groups + cap_slices - 1) / cap_slices);
  const int32_t n_slices = (n_days + per_slice - 1) / per_slice;
  DevBuf partial;
  HIP_TRY(partial.alloc(per_slice_bytes * n_slices, s));
  HIP_TRY(path_costs(f64 != 0, n_paths, path_ptr, path_link, L, link_len, speed, n_days, H_speed, dt,
                     T, per_slice, partial.as<double>(), cost, s));
  return DODE_OK;
}

dode_status dar_from_costs(const dode_routes* routes, int32_t f64, const void* Rr, const void* cost,
                           double theta, void* portions, void* W, void* stream) {
  if (!routes) return fail(DODE_ERR_ARG, "routes is NULL");
  if (!Rr || !cost || !W) return fail(DODE_ERR_ARG, "Rr, cost or W is NULL");
  if (!std::isfinite(theta)) return fail(DODE_ERR_ARG, "theta must be finite");
  hipStream_t s = as_stream(stream);
  DevBuf pi;
  HIP_TRY(pi.alloc((size_t)routes->dv.T * routes->dv.n_paths * 8, s));
  HIP_TRY(routes_rho_costs(routes->dv, f64 != 0, Rr, cost, theta, portions, W, pi.as<double>(), s));
  return DODE_OK;
}

dode_status dense_spgd_run(int32_t m, int32_t n, int32_t prec, const void* B, const void* y, void* q,
                           void* A, const int32_t* perms, int32_t E, int32_t chunk,
                           int32_t optimizer, double eta, double eps, double* loss_hist,
                           void* stream) {
  if (m < 1 || n < 1 || E < 0) return fail(DODE_ERR_SHAPE, "m=%d n=%d E=%d", m, n, E);
  if (prec < 0 || prec > 2) return fail(DODE_ERR_ARG, "prec=%d must be 0, 1 or 2", prec);
  if (chunk < 1) return fail(DODE_ERR_ARG, "chunk=%d must be positive", chunk);
  if (optimizer != 0 && optimizer != 1) return fail(DODE_ERR_ARG, "optimizer=%d", optimizer);
  if (!(eta > 0.0) || !std::isfinite(eta) || !(eps >= 0.0) || !std::isfinite(eps))
    return fail(DODE_ERR_ARG, "eta=%g eps=%g", eta, eps);
  if (!B || !y || !q || !A || (E > 0 && !perms)) return fail(DODE_ERR_ARG, "NULL array");
  if (E == 0) return DODE_OK;
  hipStream_t s = as_stream(stream);
  // every row index a kernel will use: each epoch must be a permutation of 0..m-1
  {
    std::vector<int32_t> hp((size_t)E * m);
    HIP_TRY(hipMemcpyAsync(hp.data(), perms, hp.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::vector<int32_t> seen(m, -1);
    for (int32_t e = 0; e < E; ++e)
      for (int32_t i = 0; i < m; ++i) {
        const int32_t v = hp[(size_t)e * m + i];
        if (v < 0 || v >= m || seen[v] == e)
          return fail(DODE_ERR_ARG, "perms[%d] is not a permutation of 0..m-1", e);
        seen[v] = e;
      }
  }
  const size_t ss = prec == 1 ? 8 : 4;                 // state and scratch
  const size_t bs = prec == 2 ? 2 : ss;                // one value of B
  const int32_t rows = std::min(chunk, m);
  const int32_t n_slices = (rows + dense_slice_rows() - 1) / dense_slice_rows();
  if (n_slices > 65535) return fail(DODE_ERR_SHAPE, "chunk=%d too large", chunk);
  DevBuf r, part, loss;
  HIP_TRY(r.alloc((size_t)m * ss, s));
  HIP_TRY(part.alloc((size_t)n_slices * n * ss, s));
  if (loss_hist) HIP_TRY(loss.alloc((size_t)E * 8, s));
  DenseArgs a{m, n, E, chunk, B, y, q, A, perms, r.p, part.p,
              loss_hist ? loss.as<double>() : nullptr, StepArgs{eta, eps, optimizer}};
  const bool vec = ((uintptr_t)B % 16 == 0) && ((uintptr_t)q % 16 == 0) && ((size_t)n * bs) % 16 == 0;
  HIP_TRY(prec == 2 ? dense_spgd_bf16(a, vec, s) : dense_spgd(a, prec == 1, vec, s));
  if (loss_hist) {
    HIP_TRY(hipMemcpyAsync(loss_hist, loss.p, (size_t)E * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  return DODE_OK;
}

dode_status spgd_step(const dode_dar* dar, int32_t cluster, const int32_t* chunk_h, int32_t n_h,
                      const void* X, void* Q, void* A, int32_t n_days,
                      const dode_spgd_params* params, void* stream) {
  if (dode_status st = check_dar(dar, cluster)) return st;
  if (dode_status st = check_days(n_days)) return st;
  if (dode_status st = check_params(params)) return st;
  const dode_dims& dm = dar->dims;
  if (!chunk_h || n_h < 1 || n_h > dm.H) return fail(DODE_ERR_ARG, "chunk_h must list 1..H intervals");
  if (n_days == 0) return DODE_OK;
  if (!X || !Q || !A) return fail(DODE_ERR_ARG, "X, Q or A is NULL");
  if ((int64_t)n_h * dm.L > INT32_MAX) return fail(DODE_ERR_SHAPE, "minibatch too large");
  // one permutation per cluster whose first n_h positions are the minibatch
  std::vector<int32_t> perm((size_t)dar->C * dm.H);
  std::vector<char> seen(dm.H, 0);
  for (int32_t i = 0; i < n_h; ++i) {
    if (chunk_h[i] < 0 || chunk_h[i] >= dm.H || seen[chunk_h[i]])
      return fail(DODE_ERR_ARG, "chunk_h[%d]=%d is out of range or repeated", i, chunk_h[i]);
    seen[chunk_h[i]] = 1;
  }
  for (int32_t c = 0; c < dar->C; ++c) {
    int32_t* p = perm.data() + (size_t)c * dm.H;
    int32_t k = 0;
    for (int32_t i = 0; i < n_h; ++i) p[k++] = chunk_h[i];
    for (int32_t h = 0; h < dm.H; ++h)
      if (!seen[h]) p[k++] = h;
  }
  dode_spgd_params p1 = *params;
  p1.epochs = 1;
  p1.batch_rows = n_h * dm.L;
  p1.check_finite = 0;
  if (p1.day_tile == 0) p1.day_tile = 32;   // one minibatch: nothing to tune for
  p1.refine_steps = 0;
  std::vector<int32_t> dc(n_days, cluster);
  dode_plan* raw = nullptr;
  if (dode_status st = spgd_plan_create(dar, dc.data(), n_days, &p1, perm.data(), 0, stream, &raw))
    return st;
  std::unique_ptr<dode_plan, dode_status (*)(dode_plan*)> plan(raw, spgd_plan_destroy);
  if (dode_status st = spgd_plan_load(plan.get(), X, Q, A, stream)) return st;
  if (dode_status st = run_minibatch(plan.get(), 0, 0, as_stream(stream))) return st;
  if (dode_status st = spgd_plan_store(plan.get(), Q, A, stream)) return st;
  HIP_TRY(hipStreamSynchronize(as_stream(stream)));
  return DODE_OK;
}

dode_status spgd_plan_destroy(dode_plan* plan) {
  if (!plan) return DODE_OK;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(plan->device);
  if (plan->last_stream) (void)hipStreamSynchronize(plan->last_stream);
  for (void* p : {(void*)plan->d_perm, (void*)plan->d_pos, (void*)plan->d_touched,
                  (void*)plan->d_kslot, (void*)plan->d_kdesc, (void*)plan->d_kcomp,
                  (void*)plan->d_kchunk, (void*)plan->d_kchunk_full,
                  (void*)plan->d_slabs,
                  (void*)plan->d_dc, plan->d_R, (void*)plan->d_part, (void*)plan->d_groups,
                  (void*)plan->d_full,
                  plan->d_X, plan->d_Q, plan->d_A, (void*)plan->d_loss, (void*)plan->d_order})
    if (p) (void)hipFree(p);
  free_wave_tables(plan);
  for (hipEvent_t e : plan->event_pool) (void)hipEventDestroy(e);
  if (plan->graph_exec) (void)hipGraphExecDestroy(plan->graph_exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  if (plan->capture_stream) (void)hipStreamDestroy(plan->capture_stream);
  for (hipStream_t t : plan->side_streams) (void)hipStreamDestroy(t);
  for (hipEvent_t ev : plan->slab_events) (void)hipEventDestroy(ev);
  if (plan->d_epoch) (void)hipFree(plan->d_epoch);
  if (plan->d_mb) (void)hipFree(plan->d_mb);
  if (plan->d_bar) (void)hipFree(plan->d_bar);
  (void)hipSetDevice(cur);
  delete plan;
  return DODE_OK;
}

dode_status spgd_plan_create(const dode_dar* dar, const int32_t* day_cluster, int32_t D,
                             const dode_spgd_params* params, const int32_t* perm, uint64_t seed,
                             void* stream, dode_plan** out) {
  if (!out) return fail(DODE_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!dar) return fail(DODE_ERR_ARG, "dar handle is NULL");
  if (dode_status st = check_days(D)) return st;
  if (dode_status st = check_params(params)) return st;
  if (D < 1) return fail(DODE_ERR_ARG, "a plan needs D >= 1 days");
  if (params->epochs < 1) return fail(DODE_ERR_ARG, "a plan needs epochs >= 1");
  if (!day_cluster) return fail(DODE_ERR_ARG, "day_cluster is NULL");
  for (int32_t d = 0; d < D; ++d)
    if (day_cluster[d] < 0 || day_cluster[d] >= dar->C)
      return fail(DODE_ERR_ARG, "day_cluster[%d]=%d out of range", d, day_cluster[d]);
  const dode_dims& dm = dar->dims;
  const int32_t E = params->epochs, C = dar->C;
  const int32_t bh = std::max<int32_t>(1, std::min<int32_t>(dm.H, params->batch_rows / dm.L));
  HostSched hs;
  if (dode_status st = build_sched(dm, C, E, bh, perm, seed, hs)) return st;
  std::unique_ptr<dode_plan, dode_status (*)(dode_plan*)> pl(new dode_plan(), spgd_plan_destroy);
  dode_plan* p = pl.get();
  p->dar = dar;
  p->D = D;
  p->E = E;
  p->C = C;
  p->bh = hs.bh;
  p->nch = hs.nch;
  p->mt = hs.mt;
  p->sa = StepArgs{params->eta, params->eps, params->optimizer};
  p->check_finite = params->check_finite != 0;
  HIP_TRY(hipGetDevice(&p->device));
  auto up = [&](int32_t** dst, const void* src, size_t bytes) -> hipError_t {
    hipError_t e = hipMalloc(dst, std::max<size_t>(bytes, 16));
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
  };
  HIP_TRY(up(&p->d_perm, hs.perm.data(), hs.perm.size() * 4));
  HIP_TRY(up(&p->d_pos, hs.pos.data(), hs.pos.size() * 4));
  HIP_TRY(up(&p->d_touched, hs.touched.data(), hs.touched.size() * 4));
  p->kmt = hs.mt;
  p->max_comp = hs.max_comp;
  HIP_TRY(up(&p->d_kslot, hs.kslot.data(), hs.kslot.size() * 4));
  HIP_TRY(up(&p->d_kdesc, hs.kdesc.data(), hs.kdesc.size() * 4));
  HIP_TRY(up(&p->d_kcomp, hs.kcomp.data(), hs.kcomp.size() * 4));
  p->max_chunks = hs.max_chunks;
  p->chunk_w = hs.chunk_w;
  HIP_TRY(up(&p->d_kchunk, hs.kchunk.data(), hs.kchunk.size() * 4));
  // plan day i = caller day order[i], days grouped by cluster
  std::vector<int32_t> order, dc_plan;
  p->cluster_days.assign(C, 0);
  for (int32_t c = 0; c < C; ++c)
    for (int32_t d = 0; d < D; ++d)
      if (day_cluster[d] == c) {
        order.push_back(d);
        dc_plan.push_back(c);
        ++p->cluster_days[c];
      }
  p->n_slabs = std::max<int32_t>(1, params->slabs);
  p->refine_steps = params->refine_steps;   // the work tables cover refinement steps
  p->full_chunks = p->refine_steps > 0 ? (dm.T + kChunkT - 1) / kChunkT : 0;
  if (dode_status st = set_day_groups(p, params->day_tile ? params->day_tile : 32)) return st;
  HIP_TRY(up(&p->d_order, order.data(), (size_t)D * 4));
  HIP_TRY(up(&p->d_dc, dc_plan.data(), (size_t)D * 4));
  // Plan state layout (Layout): day-blocked rows for the matrix-core path,
  // plain interval-major rows otherwise; every array carries kStatePad
  // zeroed elements past its end, and the blocked rows their zero blocks.
  // "fastest available": the matrix-core tiles need days to fill the MFMA N
  // dimension (16 per wave).  When no cluster has more than kSparseDays days
  // (one ratio matrix per day, say) the sparse kernels are faster: 1.97 vs
  // 4.83 ms per epoch with 365 one-day clusters of 50 ODs and 200 links.
  // Refinement steps need the tiles.
  const int32_t max_days = *std::max_element(p->cluster_days.begin(), p->cluster_days.end());
  if (params->kernel_path >= 2 && !dar->has_tiles)
    return fail(DODE_ERR_UNSUPPORTED, "kernel_path %d needs BF16 or FP8 storage (matrix-core tiles)",
                params->kernel_path);
  if (params->kernel_path == 3 && (params->day_tile == 0 || params->slabs > 1))
    return fail(DODE_ERR_ARG,
                "kernel_path 3 (one launch per epoch) needs a given day_tile and one day slab");
  if (params->kernel_path == 3 && params->adj_order == 2 && params->day_tile != 16)
    return fail(DODE_ERR_UNSUPPORTED,
                "kernel_path 3 runs the chunked adjoint (adj_order 2) with 16-day waves only");
  p->use_mfma = dar->has_tiles &&
                ((params->kernel_path == 0 && (max_days > kSparseDays || params->refine_steps > 0)) ||
                 params->kernel_path >= 2);
  p->one_launch = p->use_mfma && params->kernel_path == 2;
  p->persistent = p->use_mfma && params->kernel_path == 3;
  const size_t ss = state_size(dar);
  if (p->use_mfma) {
    const int64_t pb = blocked_row_blocks(dm.P), lb = blocked_row_blocks(dm.L);
    p->ly = Layout{4, pb * 4 * D, 4, lb * 4 * D, 4, lb * 4 * D, 4 * (int64_t)D, 4 * (int64_t)D,
                   4 * (int64_t)D};
  } else {
    p->ly = Layout{dm.P, (int64_t)D * dm.P, dm.L, (int64_t)D * dm.L, dm.L, (int64_t)D * dm.L, 4, 4, 4};
  }
  p->refine_steps = params->refine_steps;
  if (p->refine_steps > 0) {
    if (!p->use_mfma || !dar->has_corr)
      return fail(DODE_ERR_UNSUPPORTED,
                  "refine_steps needs FP8 storage with correction tiles and kernel_path 0, 2 or 3");
    // the whole row set as one minibatch: identity order, every departure
    // interval with every lag that stays inside the day
    std::vector<int32_t> full((size_t)2 * C * dm.H + (size_t)C * dm.T * (dm.K + 3), -1);
    for (int32_t c = 0; c < C; ++c)
      for (int32_t h = 0; h < dm.H; ++h) {
        full[(size_t)c * dm.H + h] = h;
        full[(size_t)(C + c) * dm.H + h] = h;
      }
    for (int32_t c = 0; c < C; ++c)
      for (int32_t t = 0; t < dm.T; ++t) {
        int32_t* dsc = full.data() + 2 * (size_t)C * dm.H + ((size_t)c * dm.T + t) * (dm.K + 3);
        uint64_t mask = 0;
        for (int32_t l = 0; l < dm.K; ++l) {
          const bool in = t + l < dm.H;
          dsc[kDescSlot + l] = in ? t + l : -1;
          if (in) mask |= 1ull << l;
        }
        dsc[kDescT] = t;
        dsc[kDescMask] = (int32_t)(uint32_t)mask;
        dsc[kDescMask + 1] = (int32_t)(uint32_t)(mask >> 32);
      }
    HIP_TRY(up(&p->d_full, full.data(), full.size() * 4));
    // the full batch is one component per cluster: chunks of kChunkT
    // consecutive departure intervals with the intervals h = slot that reach them
    std::vector<int32_t> fc((size_t)C * p->full_chunks * p->chunk_w, 0);
    for (int32_t c = 0; c < C; ++c)
      for (int32_t k = 0; k < p->full_chunks; ++k) {
        int32_t* ck = fc.data() + ((size_t)c * p->full_chunks + k) * p->chunk_w;
        const int32_t t0 = k * kChunkT, nt = std::min(kChunkT, dm.T - t0);
        ck[0] = t0;
        ck[1] = nt;
        int32_t nh = 0;
        for (int32_t h = t0; h <= t0 + nt - 1 + dm.K - 1 && h < dm.H; ++h, ++nh) {
          ck[3 + 2 * nh] = h;
          ck[4 + 2 * nh] = h;
        }
        ck[2] = nh;
      }
    HIP_TRY(up(&p->d_kchunk_full, fc.data(), fc.size() * 4));
  }
  const int64_t r_rows = p->refine_steps > 0 ? std::max(bh, dm.H) : bh;
  const int64_t nR = r_rows * p->ly.r_s + kStatePad, nX = dm.H * p->ly.x_h + kStatePad;
  const int64_t nQ = dm.T * p->ly.q_t + kStatePad;
  HIP_TRY(hipMalloc(&p->d_R, nR * ss));
  HIP_TRY(hipMalloc(&p->d_part, (size_t)D * dm.H * 8));
  HIP_TRY(hipMalloc(&p->d_loss, (size_t)D * 8));
  HIP_TRY(hipMalloc(&p->d_X, nX * ss));
  HIP_TRY(hipMalloc(&p->d_Q, nQ * ss));
  HIP_TRY(hipMalloc(&p->d_A, nQ * ss));
  hipStream_t s = as_stream(stream);
  HIP_TRY(fill_zero(is_f64(dar), p->d_R, nR, s));
  HIP_TRY(fill_zero(is_f64(dar), p->d_X, nX, s));
  HIP_TRY(fill_zero(is_f64(dar), p->d_Q, nQ, s));
  HIP_TRY(fill_zero(is_f64(dar), p->d_A, nQ, s));
  HIP_TRY(hipStreamSynchronize(s));
  p->tune_day_tile = p->use_mfma && params->day_tile == 0;
  p->adj_order = params->adj_order;
  p->use_graph = params->use_graph != 0;
  HIP_TRY(hipMalloc(&p->d_epoch, 16));
  HIP_TRY(set_counter(p->d_epoch, 0, s));
  HIP_TRY(hipStreamSynchronize(s));
  *out = pl.release();
  return DODE_OK;
}

dode_status spgd_plan_load(dode_plan* plan, const void* X, const void* Q, const void* A,
                           void* stream) {
  if (!plan) return fail(DODE_ERR_ARG, "plan is NULL");
  if (!X || !Q) return fail(DODE_ERR_ARG, "X or Q is NULL");
  const dode_dar* dar = plan->dar;
  const dode_dims& dm = dar->dims;
  hipStream_t s = as_stream(stream);
  const bool f64 = is_f64(dar);
  const int32_t D = plan->D;
  if (plan->check_finite)
    if (dode_status st = scan_finite(dar, X, (int64_t)D * dm.H * dm.L, s)) return st;
  const Layout& ly = plan->ly;
  HIP_TRY(gather_rows(f64, X, plan->d_X, plan->d_order, D, dm.H, dm.L, ly.x_d, ly.x_h, ly.x_b,
                      false, s));
  for (int pass = 0; pass < 2; ++pass) {
    HIP_TRY(gather_rows(f64, Q, plan->d_Q, plan->d_order, D, dm.T, dm.P, ly.q_d, ly.q_t, ly.q_b,
                        true, s));
    if (A)
      HIP_TRY(gather_rows(f64, A, plan->d_A, plan->d_order, D, dm.T, dm.P, ly.q_d, ly.q_t, ly.q_b,
                          false, s));
    else
      HIP_TRY(fill_zero(f64, plan->d_A, dm.T * ly.q_t, s));
    if (pass == 1 || !plan->tune_day_tile) break;
    // tuning runs minibatches on the loaded state; the second pass reloads it
    if (dode_status st = tune_schedule(plan, s)) return st;
    plan->tune_day_tile = false;
  }
  plan->last_stream = s;
  return DODE_OK;
}

dode_status spgd_plan_store(const dode_plan* plan, void* Q, void* A, void* stream) {
  if (!plan) return fail(DODE_ERR_ARG, "plan is NULL");
  if (!Q) return fail(DODE_ERR_ARG, "Q is NULL");
  const dode_dims& dm = plan->dar->dims;
  hipStream_t s = as_stream(stream);
  const bool f64 = is_f64(plan->dar);
  const Layout& ly = plan->ly;
  HIP_TRY(scatter_rows(f64, plan->d_Q, Q, plan->d_order, plan->D, dm.T, dm.P, ly.q_d, ly.q_t,
                       ly.q_b, s));
  if (A)
    HIP_TRY(scatter_rows(f64, plan->d_A, A, plan->d_order, plan->D, dm.T, dm.P, ly.q_d, ly.q_t,
                         ly.q_b, s));
  return DODE_OK;
}

dode_status spgd_run(dode_plan* plan, int32_t epoch_begin, int32_t n_epochs, double* loss_dev,
                     void* stream) {
  if (!plan) return fail(DODE_ERR_ARG, "plan is NULL");
  if (epoch_begin < 0 || n_epochs < 0 || epoch_begin + n_epochs > plan->E)
    return fail(DODE_ERR_ARG, "epochs [%d, %d) outside the plan's %d", epoch_begin,
                epoch_begin + n_epochs, plan->E);
  const dode_dar* dar = plan->dar;
  const dode_dims& dm = dar->dims;
  hipStream_t s = as_stream(stream);
  plan->last_stream = s;
  const int32_t D = plan->D;
  const bool graph = plan->use_graph && !plan->timing && !plan->persistent && n_epochs > 0;
  if (graph) {
    if (dode_status st = build_epoch_graph(plan)) return st;
    HIP_TRY(set_counter(plan->d_epoch, epoch_begin, s));
  }
  for (int32_t e = epoch_begin; e < epoch_begin + n_epochs; ++e) {
    if (graph) {
      HIP_TRY(hipGraphLaunch(plan->graph_exec, s));
    } else {
      if (dode_status st = run_epoch(plan, e, s)) return st;
    }
    if (loss_dev) {
      double* out = loss_dev + (size_t)(e - epoch_begin) * D;
      HIP_TRY(timed(plan, 2, s, [&] {
        hipError_t r = plain_apply_rows(dar, plan->d_dc, 0, plan->ly, plan->d_Q, plan->d_X, nullptr,
                                        plan->d_part, D, s);
        if (r == hipSuccess) r = sum_partials(plan->d_part, dm.H, D, plan->d_loss, s);
        return r != hipSuccess ? r : permute_loss(plan->d_loss, plan->d_order, D, out, s);
      }));
    }
  }
  if (plan->persistent && n_epochs > 0) {
    // a grid barrier that gave up leaves its error word set
    PersistBarrier b{};
    HIP_TRY(hipMemcpyAsync(&b, plan->d_bar, sizeof b, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (b.err)
      return fail(DODE_ERR_HIP, "persistent epoch launch: a grid barrier waited past its limit");
  }
  return DODE_OK;
}

dode_status spgd_plan_info(const dode_plan* plan, int32_t* day_tile, int32_t* n_minibatches,
                           int32_t* minibatch_intervals, int32_t* n_day_groups) {
  if (!plan) return fail(DODE_ERR_ARG, "plan is NULL");
  if (day_tile) *day_tile = plan->use_mfma ? plan->day_tile : 0;
  if (n_minibatches) *n_minibatches = plan->nch;
  if (minibatch_intervals) *minibatch_intervals = plan->bh;
  if (n_day_groups) *n_day_groups = plan->use_mfma ? plan->n_groups : 0;
  return DODE_OK;
}

dode_status spgd_plan_schedule(const dode_plan* plan, int32_t* day_tile, int32_t* adj_order,
                               int32_t* n_slabs, int32_t* n_timed, double* best_ms) {
  if (!plan) return fail(DODE_ERR_ARG, "plan is NULL");
  if (day_tile) *day_tile = plan->use_mfma ? plan->day_tile : 0;
  if (adj_order) *adj_order = plan->use_mfma ? plan->adj_order : 0;
  if (n_slabs) *n_slabs = plan->use_mfma ? plan->n_slabs : 1;
  if (n_timed) *n_timed = plan->n_timed;
  if (best_ms) *best_ms = plan->tune_ms;
  return DODE_OK;
}

dode_status spgd_plan_timing(dode_plan* plan, int32_t enable, double* ms, int64_t* launches) {
  if (!plan) return fail(DODE_ERR_ARG, "plan is NULL");
  if (plan->last_stream || plan->timing) HIP_TRY(hipStreamSynchronize(plan->last_stream));
  for (int k = 0; k < 3; ++k) {
    double tot = 0.0;
    for (auto& pr : plan->pending[k]) {
      float t = 0.f;
      HIP_TRY(hipEventElapsedTime(&t, pr.first, pr.second));
      tot += t;
    }
    if (ms) ms[k] = tot;
    if (launches) launches[k] = (int64_t)plan->pending[k].size();
    plan->pending[k].clear();
  }
  plan->event_next = 0;
  plan->timing = enable != 0;
  return DODE_OK;
}

dode_status spgd_solve(const dode_dar* dar, const int32_t* day_cluster, int32_t D, const void* X,
                       void* Q, void* A, const dode_spgd_params* params, const int32_t* perm,
                       uint64_t seed, double* loss_hist, void* stream) {
  if (!dar) return fail(DODE_ERR_ARG, "dar handle is NULL");
  if (dode_status st = check_days(D)) return st;
  if (dode_status st = check_params(params)) return st;
  if (D == 0 || params->epochs == 0) return DODE_OK;
  if (!day_cluster || !X || !Q || !A) return fail(DODE_ERR_ARG, "day_cluster, X, Q or A is NULL");
  const int32_t E = params->epochs;
  hipStream_t s = as_stream(stream);
  dode_plan* raw = nullptr;
  if (dode_status st = spgd_plan_create(dar, day_cluster, D, params, perm, seed, stream, &raw))
    return st;
  std::unique_ptr<dode_plan, dode_status (*)(dode_plan*)> plan(raw, spgd_plan_destroy);
  if (dode_status st = spgd_plan_load(plan.get(), X, Q, A, stream)) return st;
  DevBuf hist;
  if (loss_hist) HIP_TRY(hist.alloc((size_t)E * D * 8, s));
  if (dode_status st = spgd_run(plan.get(), 0, E, loss_hist ? hist.as<double>() : nullptr, stream))
    return st;
  if (dode_status st = spgd_plan_store(plan.get(), Q, A, stream)) return st;
  if (loss_hist) {
    std::vector<double> h((size_t)E * D);
    HIP_TRY(hipMemcpyAsync(h.data(), hist.p, h.size() * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int32_t d = 0; d < D; ++d)
      for (int32_t e = 0; e < E; ++e) loss_hist[(size_t)d * E + e] = h[(size_t)e * D + d];
  }
  return DODE_OK;
}

}  // extern "C"
