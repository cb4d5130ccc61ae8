// bbp.hip -- gfx950 kernels (other than the block sweeps) and the C ABI of the blockBP surface-code decoder.
//
// Data path for a batch of syndromes (one "job" = one syndrome x one coset, job = 4*syndrome + coset):
//   labels_kernel     syndrome -> f_s (left/up check chains) -> coset labels f_s L on the grid (Alg. 1)
//   init_kernel       uniform unit messages (remark 2) or given start messages, convergence flags cleared
//   sweep_kernel      block message updates, one wavefront per (job, sweep), launched per sweep class
//                     (sweep_kernel.hip, wave_sweep.hpp): Sec. III.D update, normalisation (remark 3),
//                     damping (remark 7), distance term (remark 4)
//   delta_kernel      convergence distance per job and early exit (Alg. 1 BP loop)
//   sweep_kernel      (closing mode) W_v of every block for the Bethe estimate (Lemma 3.1)
//   finalize_kernel   ln Z = sum ln W_v - sum ln <m_uv, m_vu>, decision rule, correction f_s L*
//
// The plan proves (exact rank analysis) that no boundary state can exceed bond chi for the options
// accepted here, so the compression to chi is the identity and is not executed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/bbp.h"
#include "geom.hpp"
#include "plan.hpp"
#include "bmps_launch.hpp"
#include "sweep_launch.hpp"

using bbp::SweepDesc;

namespace {

using bbp::MSTRIDE;
using bbp::SWEEP_WAVES;

thread_local std::string g_err = "no error";

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                           \
  do {                                                                                          \
    hipError_t _e = (expr);                                                                     \
    if (_e != hipSuccess) return fail(BBP_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// --------------------------------------------------------------------------------------------------
// a1/a2: syndrome -> coset labels
__global__ __launch_bounds__(256) void labels_kernel(const uint8_t* __restrict__ syn, int d, int64_t batch,
                                                     uint8_t* __restrict__ labels) {
  const int b = blockIdx.x;
  const int L = 2 * d - 1, m = 2 * d * (d - 1), nz = d * (d - 1);
  __shared__ uint8_t s[2 * 32 * 31];
  for (int i = threadIdx.x; i < m; i += blockDim.x) s[i] = syn[(int64_t)b * m + i] & 1;
  __syncthreads();
  for (int site = threadIdx.x; site < L * L; site += blockDim.x) {
    const int r = site / L, c = site % L;
    int x = 0, z = 0;
    if ((r & 1) == 0 && (c & 1) == 0) {
      for (int cc = c + 1; cc < L; cc += 2) x ^= s[(r / 2) * (d - 1) + (cc - 1) / 2];      // Z-checks right of it
      for (int rr = r + 1; rr < L; rr += 2) z ^= s[nz + ((rr - 1) / 2) * d + c / 2];        // X-checks below it
    }
    const int lx = (r == 0 && (c & 1) == 0) ? 1 : 0;   // logical X: row 0 of horizontal edges
    const int lz = (c == 0 && (r & 1) == 0) ? 1 : 0;   // logical Z: column 0 of horizontal edges
    const int bx[4] = {0, 1, 1, 0}, bz[4] = {0, 0, 1, 1};
    for (int k = 0; k < 4; ++k) {
      const int xx = x ^ (bx[k] & lx), zz = z ^ (bz[k] & lz);
      labels[((int64_t)b * 4 + k) * L * L + site] = (uint8_t)(xx | (zz << 1));
    }
  }
}

// start messages: uniform unit vectors (remark 2), or the given ones (a learned warm start) scaled to unit
// norm with the entries beyond 2^K cleared; one workgroup per job, one wavefront per message
__global__ __launch_bounds__(256) void init_kernel(float* __restrict__ msgs, const float* __restrict__ given,
                                                   const int32_t* __restrict__ edge_len, int M, int ms, int64_t jobs,
                                                   int32_t* __restrict__ conv, int32_t* __restrict__ iters,
                                                   double* __restrict__ terms) {
  const int64_t job = blockIdx.x;
  const int lane = threadIdx.x & 63;
  for (int id = threadIdx.x >> 6; id < M; id += blockDim.x >> 6) {
    const int K = edge_len[id];
    const int64_t at = (job * M + id) * ms;
    float ss = 0.0f;
    if (given) {
      for (int e = lane; e < ms; e += 64) {
        const float g = e < (1 << K) ? given[at + e] : 0.0f;
        ss += g * g;
      }
      for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o);
    }
    const bool ok = given && ss > 0.0f && ss < INFINITY;
    for (int e = lane; e < ms; e += 64) {
      const bool in = e < (1 << K);
      float v = in ? exp2f(-0.5f * K) : 0.0f;
      if (ok) v = in ? given[at + e] * __builtin_amdgcn_rsqf(ss) : 0.0f;
      msgs[at + e] = v;
    }
    if (lane == 0) terms[job * M + id] = INFINITY;   // never updated: counts as changed for a gated schedule
  }
  if (threadIdx.x == 0) {
    conv[job] = 0;
    iters[job] = 0;
  }
}

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}


__global__ void delta_kernel(const double* __restrict__ terms, int M, int64_t jobs, int32_t* __restrict__ conv,
                             int32_t* __restrict__ iters, double* __restrict__ delta, double delta0, int fixed) {
  const int64_t job = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (job >= jobs || conv[job]) return;
  double acc = 0.0;
  for (int e = 0; e < M; ++e) acc += terms[job * M + e];
  const double dl = sqrt(fmax(acc, 0.0)) / (M > 0 ? M : 1);
  delta[job] = dl;
  iters[job] += 1;
  if (!fixed && dl < delta0) conv[job] = 1;
}

__global__ __launch_bounds__(256) void finalize_kernel(const double* __restrict__ lnW, int nblocks,
                                                       const float* __restrict__ msgs, int M, int ms,
                                                       const int32_t* __restrict__ pairs, int npairs,
                                                       const uint8_t* __restrict__ labels, int d,
                                                       const double* __restrict__ delta_ws,
                                                       const int32_t* __restrict__ iters_ws, double delta1,
                                                       int rule, double* __restrict__ loglik,
                                                       double* __restrict__ delta_out,
                                                       int32_t* __restrict__ iters_out, uint8_t* __restrict__ coset,
                                                       uint8_t* __restrict__ correction) {
  const int64_t b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  __shared__ double part[4][4];
  __shared__ int badp[4][4];
  __shared__ int chosen;
  // wave k handles coset k
  {
    const int k = wid;
    const int64_t job = b * 4 + k;
    double acc = 0.0;
    int bad = 0;
    for (int blk = lane; blk < nblocks; blk += 64) {
      const double w = lnW[job * nblocks + blk];
      if (isnan(w)) bad = 1; else acc += w;
    }
    const float* mb = msgs + job * M * (int64_t)ms;
    for (int q = 0; q < npairs; ++q) {
      const float* u = mb + pairs[2 * q] * (int64_t)ms;
      const float* v = mb + pairs[2 * q + 1] * (int64_t)ms;
      double uv = 0.0;
      for (int e = lane; e < ms; e += 64) uv += (double)u[e] * (double)v[e];
      const double o = wave_sum_d(uv);
      if (o > 0.0) acc -= (lane == 0) ? log(o) : 0.0;
      else bad = 1;
    }
    acc = wave_sum_d(acc);
    for (int o = 32; o > 0; o >>= 1) bad |= __shfl_down(bad, o);
    bad = __shfl(bad, 0);
    if (lane == 0) {
      part[0][k] = acc;
      badp[0][k] = bad;
    }
  }
  __syncthreads();
  if (tid == 0) {
    double ll[4], dl[4];
    for (int k = 0; k < 4; ++k) {
      const int64_t job = b * 4 + k;
      ll[k] = badp[0][k] ? NAN : part[0][k];
      dl[k] = badp[0][k] ? INFINITY : delta_ws[job];
      loglik[job] = ll[k];
      delta_out[job] = dl[k];
      iters_out[job] = iters_ws[job];
    }
    int best = 0;
    if (rule == 1) {
      double bv = -INFINITY;
      best = 0;
      for (int k = 0; k < 4; ++k) if (!isnan(ll[k]) && ll[k] > bv) { bv = ll[k]; best = k; }
    } else {
      int any = 0;
      double bv = -INFINITY;
      for (int k = 0; k < 4; ++k)
        if (dl[k] < delta1) {
          const double v = isnan(ll[k]) ? -INFINITY : ll[k];
          if (!any || v > bv) { bv = v; best = k; }
          any = 1;
        }
      if (!any) {
        double dm = INFINITY;
        best = 0;
        for (int k = 0; k < 4; ++k) if (dl[k] < dm) { dm = dl[k]; best = k; }
      }
    }
    coset[b] = (uint8_t)best;
    chosen = best;
  }
  __syncthreads();
  const int L = 2 * d - 1, n = d * d + (d - 1) * (d - 1);
  const uint8_t* lab = labels + (b * 4 + chosen) * L * L;
  for (int site = tid; site < L * L; site += blockDim.x) {
    const int r = site / L, c = site % L;
    if ((r + c) & 1) continue;
    // qubit index: row-major over (r+c) even; rows alternate d and d-1 qubits
    const int q = (r / 2) * (2 * d - 1) + ((r & 1) ? d + (c - 1) / 2 : c / 2);
    const uint8_t lb = lab[site];
    correction[b * n + q] = (uint8_t)((lb & 1) + 2 * ((lb >> 1) & 1));
  }
}

// --------------------------------------------------------------------------------------------------
unsigned sweep_groups(int64_t jobs) { return (unsigned)((jobs + SWEEP_WAVES - 1) / SWEEP_WAVES); }

// A run of sweeps of one class inside a device sweep list: one kernel launch.
struct ClassRun {
  int cls, first, count;
  double flops;   // algorithmic flops of these sweeps for one job
};

// Sort a sweep list by class (the sweeps of one list are independent) and cut it into launches. Truncating
// sweeps, whose costs differ several-fold with their length and width, go longest first, so that the short
// ones fill the end of a launch.
std::vector<ClassRun> by_class(std::vector<SweepDesc>& v) {
  std::stable_sort(v.begin(), v.end(), [](const SweepDesc& a, const SweepDesc& b) {
    const int ca = bbp::sweep_class(a), cb = bbp::sweep_class(b);
    if (ca != cb) return ca < cb;
    return bbp::trunc_class(ca) && a.flops > b.flops;
  });
  std::vector<ClassRun> runs;
  for (int i = 0; i < (int)v.size(); ++i) {
    const int c = bbp::sweep_class(v[i]);
    if (runs.empty() || runs.back().cls != c) runs.push_back({c, i, 0, 0.0});
    runs.back().count += 1;
    runs.back().flops += v[i].flops;
  }
  return runs;
}

}  // namespace

hipError_t bbp::launch_labels(hipStream_t st, const uint8_t* syn, int d, int64_t batch, uint8_t* labels) {
  if (batch > 0) labels_kernel<<<dim3((unsigned)batch), dim3(256), 0, st>>>(syn, d, batch, labels);
  return hipGetLastError();
}

hipError_t bbp::launch_sweeps(int cls, hipStream_t st, const SweepArgs& a) {
  if (bbp::trunc_class(cls)) return launch_trunc_sweeps(st, a, (cls & 1) != 0);
  if (a.small) return launch_small_sweeps(st, a);
  bool biased = false;
  for (int k = 0; k < a.ngroups; ++k) biased |= a.g[k].biased != 0;
  if (biased && a.bf16) return hipErrorInvalidValue;   // refused earlier by resolve()
  const int variant = (cls & 15) | (a.bf16 ? 16 : 0) | (biased ? 32 : 0), kt = (cls >> 4) + 1;
  const dim3 grid(sweep_groups(a.items));
  switch (kt) {
    case 1: return launch_sweeps_k1(variant, grid, st, a);
    case 2: return launch_sweeps_k2(variant, grid, st, a);
    case 3: return launch_sweeps_k3(variant, grid, st, a);
    case 4: return launch_sweeps_k4(variant, grid, st, a);
    case 5: return launch_sweeps_k5(variant, grid, st, a);
    case 6: return launch_sweeps_k6(variant, grid, st, a);
    default: return hipErrorInvalidValue;
  }
}

namespace {

struct DevPlan {
  bbp::Plan plan;
  SweepDesc* round[2] = {nullptr, nullptr};
  SweepDesc* bethe = nullptr;
  std::vector<ClassRun> runs[3];   // rounds 0, 1 and the closing sweeps
  int32_t* edge_len = nullptr;
  int32_t* pairs = nullptr;
  int device = -1;
};

std::mutex g_mu;
std::map<std::tuple<int, int, int, int, int>, std::unique_ptr<DevPlan>> g_plans;

int validate(int32_t d, const bbp_opts* o) {
  if (!o) return fail(BBP_EINVAL, "opts is NULL");
  if (d < 2 || d > 32) return fail(BBP_EINVAL, "d must be in [2, 32]");
  if (o->block_rows < 1 || o->block_cols < 1) return fail(BBP_EINVAL, "block sizes must be >= 1");
  if (o->chi < 1) return fail(BBP_EINVAL, "chi must be >= 1");
  if (o->max_iter < 1) return fail(BBP_EINVAL, "max_iter must be >= 1");
  if (!(o->delta0 <= o->delta1)) return fail(BBP_EINVAL, "delta0 must not exceed delta1");
  if (!(o->damping >= 0.0 && o->damping < 1.0)) return fail(BBP_EINVAL, "damping must be in [0, 1)");
  if (o->rule != 0 && o->rule != 1) return fail(BBP_EINVAL, "rule must be 0 or 1");
  if (o->precision != 0 && o->precision != 1) return fail(BBP_EINVAL, "precision must be 0 (FP32) or 1 (BF16 matrix-core contractions)");
  if (o->graph != 0 && o->graph != 1) return fail(BBP_EINVAL, "graph must be 0 or 1");
  if (!(o->gate >= 0.0 && o->gate < INFINITY)) return fail(BBP_EINVAL, "gate must be finite and >= 0");
  return BBP_OK;
}

const bbp::Plan& host_plan(int d, const bbp_opts* o) { return bbp::cached_plan(d, o->block_rows, o->block_cols, o->chi); }

int device_plan(int d, const bbp_opts* o, DevPlan** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_tuple(d, o->block_rows, o->block_cols, o->chi, dev);
  auto it = g_plans.find(key);
  if (it != g_plans.end()) { *out = it->second.get(); return BBP_OK; }
  auto dp = std::make_unique<DevPlan>();
  dp->plan = host_plan(d, o);
  dp->device = dev;
  const bbp::Plan& p = dp->plan;
  for (int c = 0; c < 3; ++c) {
    std::vector<SweepDesc> v = (c < 2) ? p.round[c] : p.bethe;
    dp->runs[c] = by_class(v);
    SweepDesc*& dst = (c < 2) ? dp->round[c] : dp->bethe;
    HIP_TRY(hipMalloc(&dst, sizeof(SweepDesc) * std::max<size_t>(1, v.size())));
    if (!v.empty()) HIP_TRY(hipMemcpy(dst, v.data(), sizeof(SweepDesc) * v.size(), hipMemcpyHostToDevice));
  }
  std::vector<int32_t> el(p.edge_len.begin(), p.edge_len.end());
  if (el.empty()) el.push_back(0);
  HIP_TRY(hipMalloc(&dp->edge_len, sizeof(int32_t) * el.size()));
  HIP_TRY(hipMemcpy(dp->edge_len, el.data(), sizeof(int32_t) * el.size(), hipMemcpyHostToDevice));
  std::vector<int32_t> pr(p.pair_ids.begin(), p.pair_ids.end());
  if (pr.empty()) pr.push_back(0);
  HIP_TRY(hipMalloc(&dp->pairs, sizeof(int32_t) * pr.size()));
  HIP_TRY(hipMemcpy(dp->pairs, pr.data(), sizeof(int32_t) * pr.size(), hipMemcpyHostToDevice));
  *out = dp.get();
  g_plans.emplace(key, std::move(dp));
  return BBP_OK;
}

struct Layout {
  size_t labels, msgs, terms, lnw, conv, iters, delta, tws, total;
  int64_t tws_slots;   // items per launch of the truncating kernel (0: the plan has no truncating sweeps)
};

// Workspace slots of the truncating kernel: one per item of its largest launch, at most this many (larger
// launches run in chunks).
constexpr int64_t TRUNC_SLOTS_MAX = 32768;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

Layout layout(const bbp::Plan& p, int64_t batch) {
  const size_t jobs = (size_t)batch * 4;
  Layout l;
  size_t off = 0;
  l.labels = off; off = align256(off + jobs * p.L * p.L);
  l.msgs = off; off = align256(off + jobs * std::max(p.M, 1) * (size_t)p.mstride * sizeof(float));
  l.terms = off; off = align256(off + jobs * std::max(p.M, 1) * sizeof(double));
  l.lnw = off; off = align256(off + jobs * p.nblocks * sizeof(double));
  l.conv = off; off = align256(off + jobs * sizeof(int32_t));
  l.iters = off; off = align256(off + jobs * sizeof(int32_t));
  l.delta = off; off = align256(off + jobs * sizeof(double));
  int per_job = 0;   // largest number of truncating sweeps in one launch list
  for (int c = 0; c < 3; ++c) {
    int n = 0;
    for (const SweepDesc& s : (c < 2 ? p.round[c] : p.bethe)) n += s.trunc ? 1 : 0;
    per_job = std::max(per_job, n);
  }
  l.tws_slots = std::min<int64_t>((int64_t)jobs * per_job, TRUNC_SLOTS_MAX);
  l.tws = off; off = align256(off + (size_t)l.tws_slots * bbp::trunc_slot_bytes());
  l.total = off;
  return l;
}

struct Bbp_net_impl {
  int d;
  double p;
  std::vector<uint8_t> syndrome;
  std::vector<uint8_t> labels;   // [4][L*L]
};

// ------------------------------------------------------------------------------------------------
// Decode of a list of (d, p) groups: every sweep class of a colour round is one launch over all groups.

// Runtime launch variant, chosen by bbp_autotune per (d, blocks, chi, device).
struct Tune {
  int order = 0;     // item order inside a launch (SweepArgs::order)
  int streams = 1;   // streams over which a round's class launches are spread (1, 2 or 4)
};
std::map<std::tuple<int, int, int, int, int>, Tune> g_tune;

// Per-device auxiliary streams (default priority) and the events that fork and join them. They are shared by
// every caller on the device, so a decode that uses them enqueues (or captures) its whole work while holding
// g_aux_mu: two callers' fork / join records cannot interleave, and a capture cannot pull another caller's
// work on the auxiliary streams into its graph.
std::mutex g_aux_mu;
struct Aux {
  hipStream_t s[3] = {nullptr, nullptr, nullptr};
  hipEvent_t fork = nullptr;
  hipEvent_t join[3] = {nullptr, nullptr, nullptr};
};
std::map<int, Aux> g_aux;

int aux_for(int dev, Aux** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_aux.find(dev);
  if (it == g_aux.end()) {
    Aux a;
    for (int i = 0; i < 3; ++i) {
      HIP_TRY(hipStreamCreateWithFlags(&a.s[i], hipStreamNonBlocking));
      HIP_TRY(hipEventCreateWithFlags(&a.join[i], hipEventDisableTiming));
    }
    HIP_TRY(hipEventCreateWithFlags(&a.fork, hipEventDisableTiming));
    it = g_aux.emplace(dev, a).first;
  }
  *out = &it->second;
  return BBP_OK;
}

struct GroupRun {
  bbp_group in;
  bbp_opts opts;   // the call's options with this group's chi
  DevPlan* dp = nullptr;
  Layout lay;
  size_t off = 0;
  uint8_t* labels = nullptr;
  float* msgs = nullptr;
  double *terms = nullptr, *lnw = nullptr, *delta = nullptr;
  int32_t *conv = nullptr, *iters = nullptr;
  double* tws = nullptr;   // truncating-kernel workspace (lay.tws_slots slots)
  int64_t jobs = 0;
  int biased = 0;
};

// Validate the groups, fetch their plans and lay their state out in one workspace.
int resolve(const bbp_group* groups, int ng, const bbp_opts* opts, std::vector<GroupRun>& gr, size_t* total,
            bool need_plans) {
  if (ng < 1 || ng > bbp::MAX_GROUPS) return fail(BBP_EINVAL, "the number of groups must be in [1, 8]");
  if (!groups) return fail(BBP_EINVAL, "groups is NULL");
  gr.assign((size_t)ng, GroupRun());
  size_t off = 0;
  for (int g = 0; g < ng; ++g) {
    const bbp_group& G = groups[g];
    if (!opts) return fail(BBP_EINVAL, "opts is NULL");
    if (G.chi < 0) return fail(BBP_EINVAL, "group chi must be >= 0");
    gr[g].opts = *opts;
    if (G.chi > 0) gr[g].opts.chi = G.chi;
    int rc = validate(G.d, &gr[g].opts);
    if (rc) return rc;
    gr[g].biased = (G.noise[0] != 0.0 || G.noise[1] != 0.0 || G.noise[2] != 0.0 || G.noise[3] != 0.0) ? 1 : 0;
    if (gr[g].biased) {
      double sum = 0.0;
      for (int k = 0; k < 4; ++k) {
        if (!(G.noise[k] >= 0.0 && G.noise[k] <= 1.0)) return fail(BBP_EINVAL, "noise entries must be in [0, 1]");
        sum += G.noise[k];
      }
      if (!(G.noise[0] > 0.0) || std::fabs(sum - 1.0) > 1e-6)
        return fail(BBP_EINVAL, "noise must be probabilities summing to 1 with a positive identity entry");
      if (G.p_dev) return fail(BBP_EINVAL, "noise and p_dev are exclusive");
      if (opts->precision != 0) return fail(BBP_EUNSUPPORTED, "biased noise runs with precision 0 only");
    } else if (!G.p_dev && !(G.p > 0.0 && G.p < 1.0)) {
      return fail(BBP_EINVAL, "p must be in (0, 1)");
    }
    if (G.batch < 0) return fail(BBP_EINVAL, "batch must be >= 0");
    if (G.batch > (int64_t)1 << 24) return fail(BBP_EINVAL, "batch too large");
    gr[g].in = G;
    gr[g].lay = layout(host_plan(G.d, &gr[g].opts), G.batch);
    gr[g].off = off;
    off = align256(off + gr[g].lay.total);
    gr[g].jobs = 4 * G.batch;
    if (need_plans) {
      if ((rc = device_plan(G.d, &gr[g].opts, &gr[g].dp))) return rc;
      if (!gr[g].dp->plan.gpu_ok) return fail(BBP_EUNSUPPORTED, gr[g].dp->plan.why);
    }
  }
  *total = off;
  return BBP_OK;
}

// Timing events, reused across calls (creating two events per launch would slow the enqueue).
std::map<int, std::vector<hipEvent_t>> g_events;

int timing_event(int dev, size_t i, hipEvent_t* e) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto& v = g_events[dev];
  while (v.size() <= i) {
    hipEvent_t x;
    HIP_TRY(hipEventCreate(&x));
    v.push_back(x);
  }
  *e = v[i];
  return BBP_OK;
}

// Per-launch timing record (timing mode only).
struct Mark {
  hipEvent_t a, b;
  int kind;               // 0 other, 1 BP-round sweeps, 2 closing sweeps
  int it, cls;
  std::vector<std::pair<int, double>> work;   // (group, per-job flops of the group's sweeps of this class)
};

// Enqueue the whole decode of the groups on st (and the auxiliary streams of the tune).
int enqueue(std::vector<GroupRun>& gr, const bbp_opts* opts, const Tune& tn, hipStream_t st,
            Aux* aux, std::vector<Mark>* marks) {
  const int ng = (int)gr.size();
  // consecutive launches on one stream share their boundary event (an event record is a queue packet)
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  size_t nev = 0;
  hipEvent_t prev_end = nullptr;
  hipStream_t prev_stream = nullptr;
  auto begin_mark = [&](hipStream_t s, int kind, int it, int cls) -> int {
    if (!marks) return BBP_OK;
    Mark m;
    m.kind = kind;
    m.it = it;
    m.cls = cls;
    int rc2;
    if (prev_end && s == prev_stream) {
      m.a = prev_end;
    } else {
      if ((rc2 = timing_event(dev, nev++, &m.a))) return rc2;
      HIP_TRY(hipEventRecord(m.a, s));
    }
    if ((rc2 = timing_event(dev, nev++, &m.b))) return rc2;
    marks->push_back(m);
    return BBP_OK;
  };
  auto end_mark = [&](hipStream_t s) -> int {
    if (!marks) return BBP_OK;
    HIP_TRY(hipEventRecord(marks->back().b, s));
    prev_end = marks->back().b;
    prev_stream = s;
    return BBP_OK;
  };
  int rc;
  for (auto& g : gr) {
    if (g.in.batch == 0) continue;
    if ((rc = begin_mark(st, 0, -1, -1))) return rc;
    labels_kernel<<<dim3((unsigned)g.in.batch), dim3(256), 0, st>>>(g.in.syndromes_dev, g.in.d, g.in.batch, g.labels);
    init_kernel<<<dim3((unsigned)g.jobs), dim3(256), 0, st>>>(g.msgs, g.in.init_messages_dev, g.dp->edge_len,
                                                              g.dp->plan.M, g.dp->plan.mstride, g.jobs, g.conv,
                                                              g.iters, g.terms);
    HIP_TRY(hipGetLastError());
    if ((rc = end_mark(st))) return rc;
  }
  const int S = std::max(1, std::min(tn.streams, 4));
  auto streams_of = [&](int i) -> hipStream_t { return (i % S) == 0 ? st : aux->s[(i % S) - 1]; };
  // one colour round (list 0 / 1) or the closing sweeps (list 2): one launch per class over all groups
  auto round = [&](int list, int it) -> int {
    std::map<int, std::vector<std::pair<int, const ClassRun*>>> cls;
    for (int g = 0; g < ng; ++g)
      if (gr[g].in.batch > 0)
        for (const ClassRun& r : gr[g].dp->runs[list]) cls[r.cls].push_back({g, &r});
    if (cls.empty()) return BBP_OK;
    // largest launches first, so that the small ones fill in behind them
    std::vector<std::pair<double, int>> order;
    for (auto& kv : cls) {
      double w = 0.0;
      for (auto& gr_r : kv.second) w += (double)gr[gr_r.first].jobs * gr_r.second->flops;
      order.push_back({-w, kv.first});
    }
    std::sort(order.begin(), order.end());
    if (S > 1) {
      HIP_TRY(hipEventRecord(aux->fork, st));
      for (int i = 1; i < S; ++i) HIP_TRY(hipStreamWaitEvent(aux->s[i - 1], aux->fork, 0));
    }
    for (size_t li = 0; li < order.size(); ++li) {
      const int c = order[li].second;
      const auto& members = cls[c];
      bbp::SweepArgs sa;
      std::memset(&sa, 0, sizeof(sa));
      sa.ngroups = (int)members.size();
      sa.mode = (list == 2) ? 1 : 0;
      sa.order = tn.order;
      sa.bf16 = opts->precision == 1 ? 1 : 0;
      sa.eta = (float)opts->damping;
      sa.gate = opts->gate;
      sa.small = (opts->block_rows <= 2 && opts->block_cols <= 2 && opts->precision == 0) ? 1 : 0;
      int64_t items = 0;
      for (int k = 0; k < sa.ngroups; ++k) {
        const GroupRun& g = gr[members[k].first];
        const ClassRun& r = *members[k].second;
        bbp::SweepGroup& G = sa.g[k];
        G.sweeps = ((list == 2) ? g.dp->bethe : g.dp->round[list]) + r.first;
        G.labels = g.labels;
        G.msgs = g.msgs;
        G.terms = g.terms;
        G.conv = g.conv;
        G.lnW = g.lnw;
        G.jobs = g.jobs;
        G.item0 = items;
        G.count = r.count;
        G.d = g.in.d;
        G.M = g.dp->plan.M;
        G.nblocks = g.dp->plan.nblocks;
        G.p00 = 1.0f - (float)g.in.p;
        G.pe = (float)g.in.p / 3.0f;
        G.pdev = g.in.p_dev;
        G.biased = g.biased;
        for (int k = 0; k < 4; ++k) G.pi[k] = (float)g.in.noise[k];
        if (g.biased) {
          for (int k = 0; k < 4; ++k) G.pq[k] = g.in.noise[k];
        } else {
          G.pq[0] = 1.0 - g.in.p;
          G.pq[1] = G.pq[2] = G.pq[3] = g.in.p / 3.0;
        }
        G.mstride = g.dp->plan.mstride;
        G.chi = g.opts.chi;
        if (bbp::trunc_class(c) && !sa.tws) {
          sa.tws = g.tws;
          sa.tws_slots = g.lay.tws_slots;
        }
        items += g.jobs * (int64_t)r.count;
      }
      sa.items = items;
      hipStream_t s = streams_of((int)li);
      if ((rc = begin_mark(s, list == 2 ? 2 : 1, it, c))) return rc;
      if (marks)
        for (auto& m : members) marks->back().work.push_back({m.first, m.second->flops});
      HIP_TRY(bbp::launch_sweeps(c, s, sa));
      if ((rc = end_mark(s))) return rc;
    }
    if (S > 1) {
      for (int i = 1; i < S; ++i) {
        HIP_TRY(hipEventRecord(aux->join[i - 1], aux->s[i - 1]));
        HIP_TRY(hipStreamWaitEvent(st, aux->join[i - 1], 0));
      }
      prev_end = nullptr;
    }
    return BBP_OK;
  };
  for (int it = 0; it < opts->max_iter; ++it) {
    for (int c = 0; c < 2; ++c)
      if ((rc = round(c, it))) return rc;
    for (auto& g : gr) {
      if (g.in.batch == 0) continue;
      if ((rc = begin_mark(st, 0, it, -1))) return rc;
      delta_kernel<<<dim3((unsigned)((g.jobs + 255) / 256)), dim3(256), 0, st>>>(
          g.terms, g.dp->plan.M, g.jobs, g.conv, g.iters, g.delta, opts->delta0, opts->fixed_iters);
      HIP_TRY(hipGetLastError());
      if ((rc = end_mark(st))) return rc;
    }
  }
  if ((rc = round(2, opts->max_iter))) return rc;
  for (auto& g : gr) {
    if (g.in.batch == 0) continue;
    const bbp::Plan& P = g.dp->plan;
    if ((rc = begin_mark(st, 0, -1, -1))) return rc;
    finalize_kernel<<<dim3((unsigned)g.in.batch), dim3(256), 0, st>>>(
        g.lnw, P.nblocks, g.msgs, P.M, P.mstride, g.dp->pairs, (int)(P.pair_ids.size() / 2), g.labels, g.in.d, g.delta, g.iters,
        opts->delta1, opts->rule, g.in.loglik_dev, g.in.delta_dev, g.in.iters_dev, g.in.coset_dev,
        g.in.correction_dev);
    HIP_TRY(hipGetLastError());
    if ((rc = end_mark(st))) return rc;
  }
  for (auto& g : gr)
    if (g.in.messages_dev && g.in.batch > 0 && g.dp->plan.M > 0)
      HIP_TRY(hipMemcpyAsync(g.in.messages_dev, g.msgs, (size_t)g.jobs * g.dp->plan.M * g.dp->plan.mstride * sizeof(float),
                             hipMemcpyDeviceToDevice, st));
  return BBP_OK;
}

// Fill `timing` from the marks of a finished decode.
int collect_timing(std::vector<GroupRun>& gr, const bbp_opts* opts, std::vector<Mark>& marks, bbp_timing* timing) {
  std::memset(timing, 0, sizeof(*timing));
  // flops actually executed: a job runs the updates of iteration `it` iff it ran more than `it` iterations
  std::vector<std::vector<double>> active(gr.size());
  for (size_t g = 0; g < gr.size(); ++g) {
    active[g].assign((size_t)opts->max_iter + 1, 0.0);
    if (gr[g].in.batch == 0) continue;
    std::vector<int32_t> it_host((size_t)gr[g].jobs);
    HIP_TRY(hipMemcpy(it_host.data(), gr[g].iters, sizeof(int32_t) * gr[g].jobs, hipMemcpyDeviceToHost));
    for (auto v : it_host) active[g][std::min<int32_t>(std::max<int32_t>(v, 0), opts->max_iter)] += 1.0;
    for (int k = opts->max_iter - 1; k >= 0; --k) active[g][k] += active[g][k + 1];   // jobs with iters >= k
  }
  std::map<int, std::tuple<double, int, double>> per_class;   // class -> (ms, launches, flops)
  for (auto& m : marks) {
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, m.a, m.b));
    if (m.kind == 1) {
      double fl = 0.0;
      for (auto& w : m.work) fl += active[w.first][m.it + 1] * w.second;
      timing->update_ms += ms;
      timing->update_launches += 1;
      timing->update_flops += fl;
      auto& pc = per_class[m.cls];
      std::get<0>(pc) += ms;
      std::get<1>(pc) += 1;
      std::get<2>(pc) += fl;
    } else if (m.kind == 2) {
      timing->bethe_ms += ms;
    } else {
      timing->other_ms += ms;
    }
  }
  timing->top_class = -1;
  for (auto& kv : per_class)
    if (std::get<0>(kv.second) > timing->top_ms) {
      timing->top_class = kv.first;
      timing->top_ms = std::get<0>(kv.second);
      timing->top_launches = std::get<1>(kv.second);
      timing->top_flops = std::get<2>(kv.second);
    }
  return BBP_OK;
}

// Instantiated graphs of whole decodes, keyed by every argument that the captured work depends on. At most
// MAX_GRAPHS are kept: a new one beyond that empties the cache after a device synchronisation (no replay of
// an evicted graph can still be in flight).
std::map<std::vector<uint64_t>, hipGraphExec_t> g_graphs;
constexpr size_t MAX_GRAPHS = 64;

template <class T>
uint64_t u64(T v) {
  uint64_t r = 0;
  std::memcpy(&r, &v, std::min(sizeof(T), sizeof(r)));
  return r;
}

int decode_groups(const bbp_group* groups, int ng, const bbp_opts* opts, void* workspace, size_t workspace_bytes,
                  void* stream, bbp_timing* timing, const Tune* force) {
  std::vector<GroupRun> gr;
  size_t total = 0;
  int rc = resolve(groups, ng, opts, gr, &total, true);
  if (rc) return rc;
  if (total > 0 && !workspace) return fail(BBP_EINVAL, "workspace is NULL");
  if (workspace_bytes < total) return fail(BBP_EINVAL, "workspace too small");
  bool any = false;
  for (auto& g : gr) {
    if (g.in.batch == 0) continue;
    any = true;
    if (!g.in.syndromes_dev || !g.in.loglik_dev || !g.in.delta_dev || !g.in.iters_dev || !g.in.coset_dev ||
        !g.in.correction_dev)
      return fail(BBP_EINVAL, "a required pointer is NULL");
    char* ws = (char*)workspace + g.off;
    g.labels = (uint8_t*)(ws + g.lay.labels);
    g.msgs = (float*)(ws + g.lay.msgs);
    g.terms = (double*)(ws + g.lay.terms);
    g.lnw = (double*)(ws + g.lay.lnw);
    g.conv = (int32_t*)(ws + g.lay.conv);
    g.iters = (int32_t*)(ws + g.lay.iters);
    g.delta = (double*)(ws + g.lay.delta);
    g.tws = g.lay.tws_slots > 0 ? (double*)(ws + g.lay.tws) : nullptr;
  }
  if (!any) return BBP_OK;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  Tune tn;
  if (force) {
    tn = *force;
  } else {
    // the launch variant tuned for the group that carries the most work (jobs x flops per iteration)
    const GroupRun* big = &gr[0];
    double most = -1.0;
    for (auto& g : gr) {
      const double w = (double)g.jobs * g.dp->plan.flops_iter;
      if (w > most) {
        most = w;
        big = &g;
      }
    }
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tune.find(std::make_tuple(big->in.d, opts->block_rows, opts->block_cols, big->opts.chi, dev));
    if (it != g_tune.end()) tn = it->second;
  }
  Aux* aux = nullptr;
  if (tn.streams > 1 && (rc = aux_for(dev, &aux))) return rc;
  hipStream_t st = (hipStream_t)stream;

  std::unique_lock<std::mutex> aux_lock(g_aux_mu, std::defer_lock);
  if (aux) aux_lock.lock();
  if (timing) {
    std::vector<Mark> marks;
    rc = enqueue(gr, opts, tn, st, aux, &marks);
    if (aux) aux_lock.unlock();
    if (rc == BBP_OK) {
      if (hipStreamSynchronize(st) != hipSuccess) rc = fail(BBP_EHIP, "stream synchronisation failed");
      else rc = collect_timing(gr, opts, marks, timing);
    }
    return rc;
  }
  if (!opts->graph) return enqueue(gr, opts, tn, st, aux, nullptr);

  // graph mode: capture the decode once per argument set, replay it afterwards
  if (!st) return fail(BBP_EINVAL, "graph mode needs a stream other than the default stream");
  std::vector<uint64_t> key = {(uint64_t)dev, (uint64_t)ng, u64(workspace), (uint64_t)workspace_bytes,
                               u64(st), (uint64_t)tn.order, (uint64_t)tn.streams};
  const bbp_opts o = *opts;
  key.insert(key.end(), {(uint64_t)o.block_rows, (uint64_t)o.block_cols, (uint64_t)o.chi, (uint64_t)o.max_iter,
                         u64(o.delta0), u64(o.delta1), u64(o.damping), (uint64_t)o.rule, (uint64_t)o.fixed_iters,
                         (uint64_t)o.precision, u64(o.gate)});
  for (auto& g : gr)
    key.insert(key.end(), {(uint64_t)g.in.d, (uint64_t)g.opts.chi, u64(g.in.p), u64(g.in.p_dev),
                           u64(g.in.syndromes_dev), (uint64_t)g.in.batch,
                           u64(g.in.loglik_dev), u64(g.in.delta_dev), u64(g.in.iters_dev), u64(g.in.coset_dev),
                           u64(g.in.correction_dev), u64(g.in.init_messages_dev), u64(g.in.messages_dev),
                           u64(g.in.noise[0]), u64(g.in.noise[1]), u64(g.in.noise[2]), u64(g.in.noise[3])});
  // a cached graph is launched under the cache lock, so that no eviction can destroy it in between
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_graphs.find(key);
    if (it != g_graphs.end()) {
      HIP_TRY(hipGraphLaunch(it->second, st));
      return BBP_OK;
    }
  }
  hipGraphExec_t exec = nullptr;
  {
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    rc = enqueue(gr, opts, tn, st, aux, nullptr);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return fail(BBP_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return fail(BBP_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    if (aux) aux_lock.unlock();
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_graphs.find(key);
    if (it != g_graphs.end()) {   // another thread captured the same decode meanwhile: keep one
      (void)hipGraphExecDestroy(exec);
      exec = it->second;
    } else {
      if (g_graphs.size() >= MAX_GRAPHS) {
        HIP_TRY(hipDeviceSynchronize());
        for (auto& kv : g_graphs) (void)hipGraphExecDestroy(kv.second);
        g_graphs.clear();
      }
      g_graphs[key] = exec;
    }
    HIP_TRY(hipGraphLaunch(exec, st));
  }
  return BBP_OK;
}

// ------------------------------------------------------------------------------------------------
// Allocation-free decode (bbp_decode_device_noalloc): the workspace and the plan's device tables live in
// one static device array of BBP_SCRATCH_BYTES per device instead of caller or library allocations.
// Layout of one call: [plan tables][workspace of bbp_workspace_size], both 256-byte aligned. Every call on a
// device reuses the same array, so calls that overlap on one device race.
static __device__ __align__(256) unsigned char scratch[BBP_SCRATCH_BYTES];

// Device address of this device's copy of `scratch`, looked up once per device with that device current.
// The host-side name `scratch` is only a stand-in for the symbol; kernels and copies get this address.
std::map<int, unsigned char*> g_scratch;

int scratch_ptr(int dev, unsigned char** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_scratch.find(dev);
  if (it == g_scratch.end()) {
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(BBP_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
    it = g_scratch.emplace(dev, (unsigned char*)ptr).first;
  }
  *out = it->second;
  return BBP_OK;
}

// A plan whose device tables sit at the start of a device's scratch array: the host copies are kept for
// the life of the process, because every call enqueues their upload (another call may have overwritten
// the array since) and an enqueued copy reads its host source when it runs.
struct ScratchPlan {
  DevPlan dp;
  std::vector<SweepDesc> lists[3];
  std::vector<int32_t> edge_len, pairs;
  size_t off[5] = {0, 0, 0, 0, 0};   // byte offsets of lists 0..2, edge_len, pairs
  size_t bytes = 0;                  // total, 256-byte aligned
};
std::map<std::tuple<int, int, int, int, int>, std::unique_ptr<ScratchPlan>> g_scratch_plans;

int scratch_plan(int d, const bbp_opts* o, int dev, unsigned char* base, ScratchPlan** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_tuple(d, o->block_rows, o->block_cols, o->chi, dev);
  auto it = g_scratch_plans.find(key);
  if (it != g_scratch_plans.end()) { *out = it->second.get(); return BBP_OK; }
  auto sp = std::make_unique<ScratchPlan>();
  sp->dp.plan = host_plan(d, o);
  sp->dp.device = dev;
  const bbp::Plan& p = sp->dp.plan;
  size_t off = 0;
  for (int c = 0; c < 3; ++c) {
    sp->lists[c] = (c < 2) ? p.round[c] : p.bethe;
    sp->dp.runs[c] = by_class(sp->lists[c]);
    sp->off[c] = off;
    off = align256(off + sizeof(SweepDesc) * sp->lists[c].size());
  }
  sp->edge_len.assign(p.edge_len.begin(), p.edge_len.end());
  sp->pairs.assign(p.pair_ids.begin(), p.pair_ids.end());
  sp->off[3] = off;
  off = align256(off + sizeof(int32_t) * sp->edge_len.size());
  sp->off[4] = off;
  off = align256(off + sizeof(int32_t) * sp->pairs.size());
  sp->bytes = off;
  sp->dp.round[0] = (SweepDesc*)(base + sp->off[0]);
  sp->dp.round[1] = (SweepDesc*)(base + sp->off[1]);
  sp->dp.bethe = (SweepDesc*)(base + sp->off[2]);
  sp->dp.edge_len = (int32_t*)(base + sp->off[3]);
  sp->dp.pairs = (int32_t*)(base + sp->off[4]);
  *out = sp.get();
  g_scratch_plans.emplace(key, std::move(sp));
  return BBP_OK;
}

int decode_noalloc(int32_t d, double p, const uint8_t* syndromes_dev, int64_t batch, const bbp_opts* opts,
                   double* loglik_dev, double* delta_dev, int32_t* iters_dev, uint8_t* coset_dev,
                   uint8_t* correction_dev, void* stream) {
  if (!opts) return fail(BBP_EINVAL, "opts is NULL");
  bbp_opts o = *opts;
  o.graph = 0;   // eager launches on the caller's stream (a caller may capture them)
  bbp_group g;
  std::memset(&g, 0, sizeof(g));
  g.d = d;
  g.p = p;
  g.syndromes_dev = syndromes_dev;
  g.batch = batch;
  g.loglik_dev = loglik_dev;
  g.delta_dev = delta_dev;
  g.iters_dev = iters_dev;
  g.coset_dev = coset_dev;
  g.correction_dev = correction_dev;
  std::vector<GroupRun> gr;
  size_t total = 0;
  int rc = resolve(&g, 1, &o, gr, &total, false);
  if (rc) return rc;
  const bbp::Plan& hp = host_plan(d, &gr[0].opts);
  if (!hp.gpu_ok) return fail(BBP_EUNSUPPORTED, hp.why);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  unsigned char* base = nullptr;
  if ((rc = scratch_ptr(dev, &base))) return rc;
  ScratchPlan* sp = nullptr;
  if ((rc = scratch_plan(d, &gr[0].opts, dev, base, &sp))) return rc;
  const size_t need = sp->bytes + total;
  if (need > (size_t)BBP_SCRATCH_BYTES)
    return fail(BBP_EINVAL, "the allocation-free decode needs " + std::to_string(need) +
                                " bytes of scratch for this batch; its limit is " +
                                std::to_string((size_t)BBP_SCRATCH_BYTES) + " bytes (use bbp_decode_device)");
  if (batch == 0) return BBP_OK;
  if (!syndromes_dev || !loglik_dev || !delta_dev || !iters_dev || !coset_dev || !correction_dev)
    return fail(BBP_EINVAL, "a required pointer is NULL");
  hipStream_t st = (hipStream_t)stream;
  for (int c = 0; c < 3; ++c)
    if (!sp->lists[c].empty())
      HIP_TRY(hipMemcpyAsync(base + sp->off[c], sp->lists[c].data(), sizeof(SweepDesc) * sp->lists[c].size(),
                             hipMemcpyHostToDevice, st));
  if (!sp->edge_len.empty())
    HIP_TRY(hipMemcpyAsync(base + sp->off[3], sp->edge_len.data(), sizeof(int32_t) * sp->edge_len.size(),
                           hipMemcpyHostToDevice, st));
  if (!sp->pairs.empty())
    HIP_TRY(hipMemcpyAsync(base + sp->off[4], sp->pairs.data(), sizeof(int32_t) * sp->pairs.size(),
                           hipMemcpyHostToDevice, st));
  GroupRun& G = gr[0];
  G.dp = &sp->dp;
  unsigned char* ws = base + sp->bytes;
  G.labels = (uint8_t*)(ws + G.lay.labels);
  G.msgs = (float*)(ws + G.lay.msgs);
  G.terms = (double*)(ws + G.lay.terms);
  G.lnw = (double*)(ws + G.lay.lnw);
  G.conv = (int32_t*)(ws + G.lay.conv);
  G.iters = (int32_t*)(ws + G.lay.iters);
  G.tws = G.lay.tws_slots > 0 ? (double*)(ws + G.lay.tws) : nullptr;
  G.delta = (double*)(ws + G.lay.delta);
  Tune tn;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tune.find(std::make_tuple(d, o.block_rows, o.block_cols, G.opts.chi, dev));
    if (it != g_tune.end()) tn.order = it->second.order;
  }
  tn.streams = 1;   // auxiliary streams are not created here
  return enqueue(gr, &o, tn, st, nullptr, nullptr);
}

}  // namespace

struct bbp_net {
  Bbp_net_impl impl;
};

extern "C" {

void bbp_default_opts(bbp_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->block_rows = 6;
  o->block_cols = 6;
  o->chi = 16;
  o->max_iter = 20;
  o->delta0 = 1e-4;
  o->delta1 = 1e-2;
  o->damping = 0.1;
  o->rule = 0;
  o->fixed_iters = 0;
  o->precision = 0;
  o->graph = 0;
}

const char* bbp_last_error(void) { return g_err.c_str(); }

int bbp_build_network(int32_t d, double p, const uint8_t* syndrome, int64_t m, bbp_net** out) {
  if (!out) return fail(BBP_EINVAL, "out is NULL");
  *out = nullptr;
  if (d < 2 || d > 32) return fail(BBP_EINVAL, "d must be in [2, 32]");
  if (m != 2LL * d * (d - 1)) return fail(BBP_EINVAL, "syndrome length must be 2d(d-1)");
  if (!(p > 0.0 && p < 1.0)) return fail(BBP_EINVAL, "p must be in (0, 1)");
  if (!syndrome) return fail(BBP_EINVAL, "syndrome is NULL");
  for (int64_t i = 0; i < m; ++i)
    if (syndrome[i] > 1) return fail(BBP_EINVAL, "syndrome bytes must be 0 or 1");
  bbp_net* net = new (std::nothrow) bbp_net;
  if (!net) return fail(BBP_ENOMEM, "out of host memory");
  const int L = 2 * d - 1, nz = d * (d - 1);
  net->impl.d = d;
  net->impl.p = p;
  net->impl.syndrome.assign(syndrome, syndrome + m);
  net->impl.labels.assign((size_t)4 * L * L, 0);
  for (int r = 0; r < L; ++r)
    for (int c = 0; c < L; ++c) {
      int x = 0, z = 0;
      if ((r & 1) == 0 && (c & 1) == 0) {
        for (int cc = c + 1; cc < L; cc += 2) x ^= syndrome[(r / 2) * (d - 1) + (cc - 1) / 2];
        for (int rr = r + 1; rr < L; rr += 2) z ^= syndrome[nz + ((rr - 1) / 2) * d + c / 2];
      }
      const int lx = (r == 0 && (c & 1) == 0), lz = (c == 0 && (r & 1) == 0);
      const int bx[4] = {0, 1, 1, 0}, bz[4] = {0, 0, 1, 1};
      for (int k = 0; k < 4; ++k)
        net->impl.labels[(size_t)k * L * L + r * L + c] = (uint8_t)((x ^ (bx[k] & lx)) | ((z ^ (bz[k] & lz)) << 1));
    }
  *out = net;
  return BBP_OK;
}

int bbp_net_dims(const bbp_net* net, int32_t* d, int32_t* n, int32_t* m) {
  if (!net) return fail(BBP_EINVAL, "net is NULL");
  const int dd = net->impl.d;
  if (d) *d = dd;
  if (n) *n = dd * dd + (dd - 1) * (dd - 1);
  if (m) *m = 2 * dd * (dd - 1);
  return BBP_OK;
}

int bbp_net_labels(const bbp_net* net, uint8_t* labels) {
  if (!net || !labels) return fail(BBP_EINVAL, "NULL argument");
  std::memcpy(labels, net->impl.labels.data(), net->impl.labels.size());
  return BBP_OK;
}

void bbp_free_network(bbp_net* net) { delete net; }

int bbp_plan_query(int32_t d, const bbp_opts* opts, bbp_plan_info* info) {
  if (opts && opts->precision != 0) { /* precision does not change the plan */ }
  if (!opts) return fail(BBP_EINVAL, "opts is NULL");
  if (!info) return fail(BBP_EINVAL, "info is NULL");
  if (d < 2 || d > 32 || opts->block_rows < 1 || opts->block_cols < 1 || opts->chi < 1)
    return fail(BBP_EINVAL, "invalid d or options");
  const bbp::Plan& p = host_plan(d, opts);
  info->L = p.L;
  info->n = d * d + (d - 1) * (d - 1);
  info->m = 2 * d * (d - 1);
  info->block_grid_rows = p.nI;
  info->block_grid_cols = p.nJ;
  info->num_messages = p.M;
  info->updates_per_iter = p.M;
  info->exact_sweeps = p.exact ? 1 : 0;
  info->max_cut_rank = p.max_rank;
  info->gpu_supported = p.gpu_ok ? 1 : 0;
  info->flops_per_iter = p.flops_iter;
  info->flops_bethe = p.flops_bethe;
  info->truncating_sweeps = p.trunc_sweeps;
  info->message_stride = p.mstride;
  if (!p.gpu_ok) g_err = p.why;
  return BBP_OK;
}

int bbp_workspace_size(int32_t d, int64_t batch, const bbp_opts* opts, size_t* bytes) {
  const int rc = validate(d, opts);
  if (rc) return rc;
  if (!bytes) return fail(BBP_EINVAL, "bytes is NULL");
  if (batch < 0) return fail(BBP_EINVAL, "batch must be >= 0");
  *bytes = layout(host_plan(d, opts), batch).total;
  return BBP_OK;
}

int bbp_workspace_size_groups(const bbp_group* groups, int32_t ngroups, const bbp_opts* opts, size_t* bytes) {
  if (!bytes) return fail(BBP_EINVAL, "bytes is NULL");
  std::vector<GroupRun> gr;
  return resolve(groups, ngroups, opts, gr, bytes, false);
}

int bbp_decode_groups(const bbp_group* groups, int32_t ngroups, const bbp_opts* opts, void* workspace,
                      size_t workspace_bytes, void* stream, bbp_timing* timing) {
  return decode_groups(groups, ngroups, opts, workspace, workspace_bytes, stream, timing, nullptr);
}

int bbp_decode_device(int32_t d, double p, const uint8_t* syndromes_dev, int64_t batch, const bbp_opts* opts,
                      void* workspace, size_t workspace_bytes, double* loglik_dev, double* delta_dev,
                      int32_t* iters_dev, uint8_t* coset_dev, uint8_t* correction_dev, float* messages_dev,
                      void* stream, bbp_timing* timing) {
  bbp_group g;
  std::memset(&g, 0, sizeof(g));
  g.d = d;
  g.p = p;
  g.syndromes_dev = syndromes_dev;
  g.batch = batch;
  g.loglik_dev = loglik_dev;
  g.delta_dev = delta_dev;
  g.iters_dev = iters_dev;
  g.coset_dev = coset_dev;
  g.correction_dev = correction_dev;
  g.messages_dev = messages_dev;
  return decode_groups(&g, 1, opts, workspace, workspace_bytes, stream, timing, nullptr);
}

int bbp_decode_device_noalloc(int32_t d, double p, const uint8_t* syndromes_dev, int64_t batch,
                              const bbp_opts* opts, double* loglik_dev, double* delta_dev, int32_t* iters_dev,
                              uint8_t* coset_dev, uint8_t* correction_dev, void* stream) {
  return decode_noalloc(d, p, syndromes_dev, batch, opts, loglik_dev, delta_dev, iters_dev, coset_dev,
                        correction_dev, stream);
}

int bbp_noalloc_max_batch(int32_t d, const bbp_opts* opts, int64_t* max_batch) {
  int rc = validate(d, opts);
  if (rc) return rc;
  if (!max_batch) return fail(BBP_EINVAL, "max_batch is NULL");
  const bbp::Plan& p = host_plan(d, opts);
  size_t tab = 0;
  tab = align256(tab + sizeof(SweepDesc) * p.round[0].size());
  tab = align256(tab + sizeof(SweepDesc) * p.round[1].size());
  tab = align256(tab + sizeof(SweepDesc) * p.bethe.size());
  tab = align256(tab + sizeof(int32_t) * p.edge_len.size());
  tab = align256(tab + sizeof(int32_t) * p.pair_ids.size());
  int64_t lo = 0, hi = (int64_t)1 << 24;
  while (lo < hi) {   // largest batch whose tables and workspace fit
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (tab + layout(p, mid).total <= (size_t)BBP_SCRATCH_BYTES) lo = mid;
    else hi = mid - 1;
  }
  *max_batch = lo;
  return BBP_OK;
}

// ---- boundary-MPS decoder (single block) ----
static int bmps_check(int32_t d, int64_t batch, int32_t chi) {
  if (d < 2 || d > 32) return fail(BBP_EINVAL, "d must be in [2, 32]");
  if (chi < 1 || chi > bbp::BMPS_CHI_MAX) return fail(BBP_EINVAL, "chi must be in [1, 16]");
  if (batch < 0) return fail(BBP_EINVAL, "batch must be >= 0");
  if (batch > (int64_t)1 << 22) return fail(BBP_EINVAL, "batch too large");
  return BBP_OK;
}

static size_t bmps_label_bytes(int32_t d, int64_t batch) {
  const int64_t L = 2 * d - 1;
  return align256((size_t)(batch * 4 * L * L));
}

int bbp_bmps_workspace_size(int32_t d, int64_t batch, int32_t chi, size_t* bytes) {
  int rc = bmps_check(d, batch, chi);
  if (rc) return rc;
  if (!bytes) return fail(BBP_EINVAL, "bytes is NULL");
  *bytes = bmps_label_bytes(d, batch) + align256(bbp::bmps_state_bytes(d, 4 * batch));
  return BBP_OK;
}

int bbp_bmps_decode_device(int32_t d, double p, const double* p_dev, const double* noise,
                           const uint8_t* syndromes_dev, int64_t batch, int32_t chi, void* workspace,
                           size_t workspace_bytes, double* loglik_dev, uint8_t* coset_dev, uint8_t* correction_dev,
                           void* stream, float* kernel_ms) {
  int rc = bmps_check(d, batch, chi);
  if (rc) return rc;
  bbp::BmpsArgs a;
  std::memset(&a, 0, sizeof(a));
  if (noise) {
    double sum = 0.0;
    for (int k = 0; k < 4; ++k) {
      if (!(noise[k] >= 0.0 && noise[k] <= 1.0)) return fail(BBP_EINVAL, "noise entries must be in [0, 1]");
      sum += noise[k];
      a.pi[k] = noise[k];
    }
    if (!(noise[0] > 0.0) || std::fabs(sum - 1.0) > 1e-6)
      return fail(BBP_EINVAL, "noise must be probabilities summing to 1 with a positive identity entry");
    if (p_dev) return fail(BBP_EINVAL, "noise and p_dev are exclusive");
    a.biased = 1;
  } else if (!p_dev && !(p > 0.0 && p < 1.0)) {
    return fail(BBP_EINVAL, "p must be in (0, 1)");
  }
  if (kernel_ms) *kernel_ms = 0.0f;
  if (batch == 0) return BBP_OK;
  if (!syndromes_dev || !workspace || !loglik_dev || !coset_dev) return fail(BBP_EINVAL, "NULL device pointer");
  size_t need = 0;
  bbp_bmps_workspace_size(d, batch, chi, &need);
  if (workspace_bytes < need) return fail(BBP_EINVAL, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  uint8_t* base = (uint8_t*)workspace;
  const size_t lb = bmps_label_bytes(d, batch);
  const int64_t L = 2 * d - 1, jobs = 4 * batch;
  a.labels = base;
  a.A = (double*)(base + lb);
  a.Q = a.A + jobs * L * (16 * 2 * 16);
  a.loglik = loglik_dev;
  a.pdev = p_dev;
  a.d = d;
  a.chi = chi;
  a.jobs = jobs;
  a.p00 = 1.0 - p;
  a.pe = p / 3.0;
  HIP_TRY(bbp::launch_labels(st, syndromes_dev, d, batch, base));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (kernel_ms) {
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, st));
  }
  HIP_TRY(bbp::launch_bmps_contract(st, a));
  if (kernel_ms) HIP_TRY(hipEventRecord(e1, st));
  HIP_TRY(bbp::launch_bmps_decide(st, a, coset_dev, correction_dev));
  if (kernel_ms) {
    HIP_TRY(hipEventSynchronize(e1));
    HIP_TRY(hipEventElapsedTime(kernel_ms, e0, e1));
    HIP_TRY(hipEventDestroy(e0));
    HIP_TRY(hipEventDestroy(e1));
  }
  return BBP_OK;
}

int bbp_set_tuning(int32_t d, const bbp_opts* opts, const bbp_tuning* t) {
  int rc = validate(d, opts);
  if (rc) return rc;
  if (!t || (t->order != 0 && t->order != 1) || (t->streams != 1 && t->streams != 2 && t->streams != 4))
    return fail(BBP_EINVAL, "tuning must have order 0 or 1 and 1, 2 or 4 streams");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  Tune tn;
  tn.order = t->order;
  tn.streams = t->streams;
  g_tune[std::make_tuple(d, opts->block_rows, opts->block_cols, opts->chi, dev)] = tn;
  return BBP_OK;
}

int bbp_autotune(int32_t d, double p, const uint8_t* syndromes_dev, int64_t batch, const bbp_opts* opts,
                 void* workspace, size_t workspace_bytes, void* stream, bbp_tuning* best) {
  int rc = validate(d, opts);
  if (rc) return rc;
  if (!best) return fail(BBP_EINVAL, "best is NULL");
  if (batch < 1) return fail(BBP_EINVAL, "autotuning needs a batch of at least one syndrome");
  const int n = d * d + (d - 1) * (d - 1);
  void* out = nullptr;
  const size_t outb = (size_t)batch * (4 * 8 + 4 * 8 + 4 * 4 + 1 + n) + 64;
  if (hipMalloc(&out, outb) != hipSuccess) return fail(BBP_ENOMEM, "device allocation failed");
  bbp_group g;
  std::memset(&g, 0, sizeof(g));
  g.d = d;
  g.p = p;
  g.syndromes_dev = syndromes_dev;
  g.batch = batch;
  g.loglik_dev = (double*)out;
  g.delta_dev = g.loglik_dev + batch * 4;
  g.iters_dev = (int32_t*)(g.delta_dev + batch * 4);
  g.coset_dev = (uint8_t*)(g.iters_dev + batch * 4);
  g.correction_dev = g.coset_dev + batch;
  bbp_opts o = *opts;
  o.graph = 0;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  Tune pick;
  double best_ms = -1.0;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = fail(BBP_EHIP, "event");
  const int orders[2] = {0, 1}, streams[3] = {1, 2, 4};
  for (int oi = 0; oi < 2 && rc == BBP_OK; ++oi)
    for (int si = 0; si < 3 && rc == BBP_OK; ++si) {
      Tune tn;
      tn.order = orders[oi];
      tn.streams = streams[si];
      rc = decode_groups(&g, 1, &o, workspace, workspace_bytes, st, nullptr, &tn);   // warm-up
      if (rc) break;
      if (hipEventRecord(e0, st) != hipSuccess) { rc = fail(BBP_EHIP, "event record"); break; }
      for (int rep = 0; rep < 2 && rc == BBP_OK; ++rep)
        rc = decode_groups(&g, 1, &o, workspace, workspace_bytes, st, nullptr, &tn);
      if (rc) break;
      float ms = 0.0f;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        rc = fail(BBP_EHIP, "timing failed");
        break;
      }
      if (best_ms < 0.0 || ms / 2.0 < best_ms) {
        best_ms = ms / 2.0;
        pick = tn;
      }
    }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  (void)hipFree(out);
  if (rc) return rc;
  best->order = pick.order;
  best->streams = pick.streams;
  best->ms = best_ms;
  return bbp_set_tuning(d, opts, best);
}

int bbp_blockbp_decode(bbp_net* const* nets, int64_t batch, const bbp_opts* opts, double* loglik, double* delta,
                       int32_t* iters, uint8_t* coset, uint8_t* correction) {
  if (batch <= 0) return batch == 0 ? BBP_OK : fail(BBP_EINVAL, "batch must be >= 0");
  if (!nets) return fail(BBP_EINVAL, "nets is NULL");
  if (!loglik || !delta || !iters || !coset || !correction) return fail(BBP_EINVAL, "a required pointer is NULL");
  // group the networks by (d, p), keeping each group's members in input order
  std::vector<std::pair<int, double>> keys;
  std::vector<std::vector<int64_t>> members;
  int nmax = 0;
  for (int64_t i = 0; i < batch; ++i) {
    if (!nets[i]) return fail(BBP_EINVAL, "a network is NULL");
    const int d = nets[i]->impl.d;
    const double p = nets[i]->impl.p;
    nmax = std::max(nmax, d * d + (d - 1) * (d - 1));
    size_t k = 0;
    while (k < keys.size() && !(keys[k].first == d && keys[k].second == p)) ++k;
    if (k == keys.size()) {
      if ((int)keys.size() == bbp::MAX_GROUPS) return fail(BBP_EINVAL, "at most 8 distinct (d, p) per call");
      keys.push_back({d, p});
      members.emplace_back();
    }
    members[k].push_back(i);
  }
  const int ng = (int)keys.size();
  std::vector<bbp_group> groups((size_t)ng);
  std::memset(groups.data(), 0, sizeof(bbp_group) * groups.size());
  std::vector<std::vector<uint8_t>> syn((size_t)ng);
  size_t out_bytes = 0, syn_bytes = 0;
  std::vector<size_t> out_off((size_t)ng), syn_off((size_t)ng);
  for (int g = 0; g < ng; ++g) {
    const int d = keys[g].first, m = 2 * d * (d - 1), n = d * d + (d - 1) * (d - 1);
    const int64_t b = (int64_t)members[g].size();
    syn[g].resize((size_t)b * m);
    for (int64_t j = 0; j < b; ++j)
      std::memcpy(&syn[g][(size_t)j * m], nets[members[g][j]]->impl.syndrome.data(), m);
    syn_off[g] = syn_bytes;
    syn_bytes = align256(syn_bytes + syn[g].size());
    out_off[g] = out_bytes;
    out_bytes = align256(out_bytes + (size_t)b * (4 * 8 + 4 * 8 + 4 * 4 + 1 + n));
    groups[g].d = d;
    groups[g].p = keys[g].second;
    groups[g].batch = b;
  }
  size_t wsb = 0;
  int rc = bbp_workspace_size_groups(groups.data(), ng, opts, &wsb);
  if (rc) return rc;
  void *ws = nullptr, *dsyn = nullptr, *dout = nullptr;
  auto cleanup = [&]() { if (ws) (void)hipFree(ws); if (dsyn) (void)hipFree(dsyn); if (dout) (void)hipFree(dout); };
  if (hipMalloc(&ws, std::max<size_t>(wsb, 256)) != hipSuccess || hipMalloc(&dsyn, syn_bytes) != hipSuccess ||
      hipMalloc(&dout, out_bytes) != hipSuccess) {
    cleanup();
    return fail(BBP_ENOMEM, "device allocation failed");
  }
  for (int g = 0; g < ng; ++g) {
    const int64_t b = groups[g].batch;
    char* o = (char*)dout + out_off[g];
    groups[g].syndromes_dev = (const uint8_t*)((char*)dsyn + syn_off[g]);
    groups[g].loglik_dev = (double*)o;
    groups[g].delta_dev = groups[g].loglik_dev + b * 4;
    groups[g].iters_dev = (int32_t*)(groups[g].delta_dev + b * 4);
    groups[g].coset_dev = (uint8_t*)(groups[g].iters_dev + b * 4);
    groups[g].correction_dev = groups[g].coset_dev + b;
    if (hipMemcpy((void*)groups[g].syndromes_dev, syn[g].data(), syn[g].size(), hipMemcpyHostToDevice) != hipSuccess) {
      cleanup();
      return fail(BBP_EHIP, "copy of syndromes failed");
    }
  }
  bbp_opts o = *opts;
  o.graph = 0;
  rc = decode_groups(groups.data(), ng, &o, ws, wsb, nullptr, nullptr, nullptr);
  if (rc == BBP_OK && hipDeviceSynchronize() != hipSuccess) rc = fail(BBP_EHIP, "decode failed");
  std::memset(correction, 0, (size_t)batch * nmax);
  for (int g = 0; g < ng && rc == BBP_OK; ++g) {
    const int d = groups[g].d, n = d * d + (d - 1) * (d - 1);
    const int64_t b = groups[g].batch;
    std::vector<double> ll((size_t)b * 4), dl((size_t)b * 4);
    std::vector<int32_t> it((size_t)b * 4);
    std::vector<uint8_t> cs((size_t)b), corr((size_t)b * n);
    if (hipMemcpy(ll.data(), groups[g].loglik_dev, b * 32, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(dl.data(), groups[g].delta_dev, b * 32, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(it.data(), groups[g].iters_dev, b * 16, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(cs.data(), groups[g].coset_dev, b, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(corr.data(), groups[g].correction_dev, (size_t)b * n, hipMemcpyDeviceToHost) != hipSuccess) {
      rc = fail(BBP_EHIP, "copy back failed");
      break;
    }
    for (int64_t j = 0; j < b; ++j) {
      const int64_t i = members[g][j];
      for (int k = 0; k < 4; ++k) {
        loglik[i * 4 + k] = ll[j * 4 + k];
        delta[i * 4 + k] = dl[j * 4 + k];
        iters[i * 4 + k] = it[j * 4 + k];
      }
      coset[i] = cs[j];
      std::memcpy(correction + (size_t)i * nmax, &corr[(size_t)j * n], n);
    }
  }
  cleanup();
  return rc;
}

int bbp_reference_update_host(int32_t d, double p, const bbp_opts* opts, const uint8_t* labels, int32_t msg_id,
                              const double* msgs, double* out, double* logscale) {
  if (!opts || !labels || !msgs || !out || !logscale) return fail(BBP_EINVAL, "NULL argument");
  if (d < 2 || d > 32 || opts->block_rows < 1 || opts->block_cols < 1 || opts->chi < 1)
    return fail(BBP_EINVAL, "invalid d or options");
  const bbp::Plan& P = host_plan(d, opts);
  const SweepDesc* found = nullptr;
  if (msg_id >= 0) {
    for (int c = 0; c < 2; ++c)
      for (auto& s : P.round[c]) if (s.msg_out == msg_id) found = &s;
  } else if (-1 - msg_id < (int)P.bethe.size()) {
    found = &P.bethe[-1 - msg_id];
  }
  if (!found) return fail(BBP_EINVAL, "unknown message or block id");
  const float eps = (float)p;
  const float pi[4] = {1.0f - eps, eps / 3.0f, eps / 3.0f, eps / 3.0f};
  return bbp::host_sweep(P, *found, labels, pi, msgs, out, logscale);
}

}  // extern "C"
