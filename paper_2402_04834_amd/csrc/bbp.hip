// bbp.hip -- gfx950 kernels (other than the block sweeps) and the C ABI of the blockBP surface-code decoder.
//
// Data path for a batch of syndromes (one "job" = one syndrome x one coset, job = 4*syndrome + coset):
//   labels_kernel     syndrome -> f_s (left/up check chains) -> coset labels f_s L on the grid (Alg. 1)
//   init_kernel       uniform unit messages (remark 2), convergence flags cleared
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

__global__ void init_kernel(float* __restrict__ msgs, const int32_t* __restrict__ edge_len, int M, int64_t jobs,
                            int32_t* __restrict__ conv, int32_t* __restrict__ iters) {
  const int64_t job = blockIdx.x;
  for (int e = threadIdx.x; e < M * MSTRIDE; e += blockDim.x) {
    const int id = e / MSTRIDE, h = e % MSTRIDE;
    const int K = edge_len[id];
    msgs[job * M * MSTRIDE + e] = (h < (1 << K)) ? exp2f(-0.5f * K) : 0.0f;
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
                                                       const float* __restrict__ msgs, int M,
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
    const float* mb = msgs + job * M * MSTRIDE;
    for (int q = 0; q < npairs; ++q) {
      const float* u = mb + pairs[2 * q] * MSTRIDE;
      const float* v = mb + pairs[2 * q + 1] * MSTRIDE;
      const double o = wave_sum_d((double)u[lane] * (double)v[lane]);
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

// Sort a sweep list by class (the sweeps of one list are independent) and cut it into launches.
std::vector<ClassRun> by_class(std::vector<SweepDesc>& v) {
  std::stable_sort(v.begin(), v.end(),
                   [](const SweepDesc& a, const SweepDesc& b) { return bbp::sweep_class(a) < bbp::sweep_class(b); });
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

hipError_t bbp::launch_sweeps(int cls, unsigned count, hipStream_t st, const SweepArgs& a) {
  const int variant = cls & 15, kt = (cls >> 4) + 1;
  const dim3 grid(sweep_groups(a.jobs), count);
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
  if (o->precision != 0) return fail(BBP_EUNSUPPORTED, "only precision 0 (FP32) is implemented");
  return BBP_OK;
}

const bbp::Plan& host_plan(int d, const bbp_opts* o) {
  static std::map<std::tuple<int, int, int, int>, bbp::Plan> cache;
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_tuple(d, o->block_rows, o->block_cols, o->chi);
  auto it = cache.find(key);
  if (it == cache.end()) it = cache.emplace(key, bbp::make_plan(d, o->block_rows, o->block_cols, o->chi)).first;
  return it->second;
}

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
  size_t labels, msgs, terms, lnw, conv, iters, delta, total;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

Layout layout(const bbp::Plan& p, int64_t batch) {
  const size_t jobs = (size_t)batch * 4;
  Layout l;
  size_t off = 0;
  l.labels = off; off = align256(off + jobs * p.L * p.L);
  l.msgs = off; off = align256(off + jobs * std::max(p.M, 1) * MSTRIDE * sizeof(float));
  l.terms = off; off = align256(off + jobs * std::max(p.M, 1) * sizeof(double));
  l.lnw = off; off = align256(off + jobs * p.nblocks * sizeof(double));
  l.conv = off; off = align256(off + jobs * sizeof(int32_t));
  l.iters = off; off = align256(off + jobs * sizeof(int32_t));
  l.delta = off; off = align256(off + jobs * sizeof(double));
  l.total = off;
  return l;
}

struct Bbp_net_impl {
  int d;
  double p;
  std::vector<uint8_t> syndrome;
  std::vector<uint8_t> labels;   // [4][L*L]
};

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
  info->max_boundary_rank = p.max_rank;
  info->gpu_supported = p.gpu_ok ? 1 : 0;
  info->flops_per_iter = p.flops_iter;
  info->flops_bethe = p.flops_bethe;
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

int bbp_decode_device(int32_t d, double p, const uint8_t* syndromes_dev, int64_t batch, const bbp_opts* opts,
                      void* workspace, size_t workspace_bytes, double* loglik_dev, double* delta_dev,
                      int32_t* iters_dev, uint8_t* coset_dev, uint8_t* correction_dev, float* messages_dev,
                      void* stream, bbp_timing* timing) {
  int rc = validate(d, opts);
  if (rc) return rc;
  if (!(p > 0.0 && p < 1.0)) return fail(BBP_EINVAL, "p must be in (0, 1)");
  if (batch < 0) return fail(BBP_EINVAL, "batch must be >= 0");
  if (batch == 0) return BBP_OK;
  if (batch > (int64_t)1 << 24) return fail(BBP_EINVAL, "batch too large");
  if (!syndromes_dev || !workspace || !loglik_dev || !delta_dev || !iters_dev || !coset_dev || !correction_dev)
    return fail(BBP_EINVAL, "a required pointer is NULL");
  DevPlan* dp = nullptr;
  rc = device_plan(d, opts, &dp);
  if (rc) return rc;
  const bbp::Plan& P = dp->plan;
  if (!P.gpu_ok) return fail(BBP_EUNSUPPORTED, P.why);
  const Layout lay = layout(P, batch);
  if (workspace_bytes < lay.total) return fail(BBP_EINVAL, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  uint8_t* labels = (uint8_t*)(ws + lay.labels);
  float* msgs = (float*)(ws + lay.msgs);
  double* terms = (double*)(ws + lay.terms);
  double* lnw = (double*)(ws + lay.lnw);
  int32_t* conv = (int32_t*)(ws + lay.conv);
  int32_t* iters = (int32_t*)(ws + lay.iters);
  double* delta = (double*)(ws + lay.delta);
  const int64_t jobs = batch * 4;
  const float eps = (float)p;
  const float pi0 = 1.0f - eps, pe = eps / 3.0f;

  std::vector<hipEvent_t> evs;
  auto mark = [&]() -> int {
    if (!timing) return BBP_OK;
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    HIP_TRY(hipEventRecord(e, st));
    evs.push_back(e);
    return BBP_OK;
  };
  std::vector<int> kinds;   // kind of the interval ending at each mark: 0 other, 1 update, 2 bethe

  if ((rc = mark())) return rc;
  labels_kernel<<<dim3((unsigned)batch), dim3(256), 0, st>>>(syndromes_dev, d, batch, labels);
  init_kernel<<<dim3((unsigned)jobs), dim3(256), 0, st>>>(msgs, dp->edge_len, P.M, jobs, conv, iters);
  HIP_TRY(hipGetLastError());
  if ((rc = mark())) return rc;
  kinds.push_back(0);
  bbp::SweepArgs sa;
  sa.d = d;
  sa.labels = labels;
  sa.msgs = msgs;
  sa.M = P.M;
  sa.terms = terms;
  sa.conv = conv;
  sa.p00 = pi0;
  sa.pe = pe;
  sa.eta = (float)opts->damping;
  sa.lnW = lnw;
  sa.nblocks = P.nblocks;
  sa.jobs = jobs;
  std::vector<std::pair<int, const ClassRun*>> upd;   // (iteration, run) of each update interval
  for (int it = 0; it < opts->max_iter; ++it) {
    for (int c = 0; c < 2; ++c) {
      for (const ClassRun& r : dp->runs[c]) {
        sa.sweeps = dp->round[c] + r.first;
        sa.mode = 0;
        HIP_TRY(bbp::launch_sweeps(r.cls, (unsigned)r.count, st, sa));
        if ((rc = mark())) return rc;
        kinds.push_back(1);
        upd.emplace_back(it, &r);
      }
    }
    delta_kernel<<<dim3((unsigned)((jobs + 255) / 256)), dim3(256), 0, st>>>(terms, P.M, jobs, conv, iters, delta,
                                                                            opts->delta0, opts->fixed_iters);
    HIP_TRY(hipGetLastError());
    if ((rc = mark())) return rc;
    kinds.push_back(0);
  }
  for (const ClassRun& r : dp->runs[2]) {
    sa.sweeps = dp->bethe + r.first;
    sa.mode = 1;
    HIP_TRY(bbp::launch_sweeps(r.cls, (unsigned)r.count, st, sa));
  }
  if ((rc = mark())) return rc;
  kinds.push_back(2);
  finalize_kernel<<<dim3((unsigned)batch), dim3(256), 0, st>>>(
      lnw, P.nblocks, msgs, P.M, dp->pairs, (int)(P.pair_ids.size() / 2), labels, d, delta, iters, opts->delta1,
      opts->rule, loglik_dev, delta_dev, iters_dev, coset_dev, correction_dev);
  HIP_TRY(hipGetLastError());
  if (messages_dev)
    HIP_TRY(hipMemcpyAsync(messages_dev, msgs, (size_t)jobs * P.M * MSTRIDE * sizeof(float),
                           hipMemcpyDeviceToDevice, st));
  if ((rc = mark())) return rc;
  kinds.push_back(0);

  if (timing) {
    HIP_TRY(hipStreamSynchronize(st));
    std::memset(timing, 0, sizeof(*timing));
    // flops actually executed: a job runs the updates of iteration `it` iff it ran more than `it` iterations
    std::vector<int32_t> it_host((size_t)jobs);
    HIP_TRY(hipMemcpy(it_host.data(), iters, sizeof(int32_t) * jobs, hipMemcpyDeviceToHost));
    std::vector<double> active((size_t)opts->max_iter + 1, 0.0);
    for (auto v : it_host) active[std::min<int32_t>(std::max<int32_t>(v, 0), opts->max_iter)] += 1.0;
    for (int k = opts->max_iter - 1; k >= 0; --k) active[k] += active[k + 1];   // jobs with iters >= k
    std::map<int, std::tuple<double, int, double>> per_class;   // class -> (ms, launches, flops)
    size_t u = 0;
    for (size_t k = 1; k < evs.size(); ++k) {
      float ms = 0.0f;
      HIP_TRY(hipEventElapsedTime(&ms, evs[k - 1], evs[k]));
      const int kind = kinds[k - 1];
      if (kind == 1) {
        const int it = upd[u].first;
        const ClassRun* r = upd[u].second;
        ++u;
        const double fl = active[it + 1] * r->flops;
        timing->update_ms += ms;
        timing->update_launches += 1;
        timing->update_flops += fl;
        auto& pc = per_class[r->cls];
        std::get<0>(pc) += ms;
        std::get<1>(pc) += 1;
        std::get<2>(pc) += fl;
      } else if (kind == 2) {
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
    for (auto e : evs) (void)hipEventDestroy(e);
  }
  return BBP_OK;
}

int bbp_blockbp_decode(bbp_net* const* nets, int64_t batch, const bbp_opts* opts, double* loglik, double* delta,
                       int32_t* iters, uint8_t* coset, uint8_t* correction) {
  if (batch <= 0) return batch == 0 ? BBP_OK : fail(BBP_EINVAL, "batch must be >= 0");
  if (!nets || !nets[0]) return fail(BBP_EINVAL, "nets is NULL");
  if (!loglik || !delta || !iters || !coset || !correction) return fail(BBP_EINVAL, "a required pointer is NULL");
  const int d = nets[0]->impl.d;
  const double p = nets[0]->impl.p;
  for (int64_t i = 0; i < batch; ++i)
    if (!nets[i] || nets[i]->impl.d != d || nets[i]->impl.p != p)
      return fail(BBP_EINVAL, "all networks of one call must share d and p");
  const int m = 2 * d * (d - 1), n = d * d + (d - 1) * (d - 1);
  size_t wsb = 0;
  int rc = bbp_workspace_size(d, batch, opts, &wsb);
  if (rc) return rc;
  std::vector<uint8_t> syn((size_t)batch * m);
  for (int64_t i = 0; i < batch; ++i) std::memcpy(&syn[(size_t)i * m], nets[i]->impl.syndrome.data(), m);
  void *ws = nullptr, *dsyn = nullptr, *dout = nullptr;
  const size_t outb = (size_t)batch * (4 * 8 + 4 * 8 + 4 * 4 + 1 + n);
  auto cleanup = [&]() { if (ws) (void)hipFree(ws); if (dsyn) (void)hipFree(dsyn); if (dout) (void)hipFree(dout); };
  if (hipMalloc(&ws, wsb) != hipSuccess || hipMalloc(&dsyn, syn.size()) != hipSuccess ||
      hipMalloc(&dout, outb) != hipSuccess) {
    cleanup();
    return fail(BBP_ENOMEM, "device allocation failed");
  }
  char* o = (char*)dout;
  double* dl = (double*)o;
  double* dd = dl + batch * 4;
  int32_t* di = (int32_t*)(dd + batch * 4);
  uint8_t* dc = (uint8_t*)(di + batch * 4);
  uint8_t* dcorr = dc + batch;
  if (hipMemcpy(dsyn, syn.data(), syn.size(), hipMemcpyHostToDevice) != hipSuccess) {
    cleanup();
    return fail(BBP_EHIP, "copy of syndromes failed");
  }
  rc = bbp_decode_device(d, p, (const uint8_t*)dsyn, batch, opts, ws, wsb, dl, dd, di, dc, dcorr, nullptr, nullptr,
                         nullptr);
  if (rc == BBP_OK) {
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(loglik, dl, batch * 4 * 8, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(delta, dd, batch * 4 * 8, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(iters, di, batch * 4 * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(coset, dc, batch, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(correction, dcorr, (size_t)batch * n, hipMemcpyDeviceToHost) != hipSuccess)
      rc = fail(BBP_EHIP, "decode or copy back failed");
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
