// Host runtime of libbpdc: the C ABI of include/bpdc.h.
//
// Responsibilities: validation of codes and parameters, the prior-LLR
// conversion, device copies of the Tanner graph (CSR + CSC) and of the
// degeneracy matrix, plans (which kernel family decodes which code, the
// autotuned tile, the code-specialised lane kernels compiled with hipRTC and
// cached on disk), workspace sizing, dispatch on the caller's stream, HIP
// graph capture of the multi-code launch, and the thread-local error state.
#include "../../include/bpdc.h"

#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "lane_spec.h"

// Source of the lane kernel (bpdc_device.h + lane_kernel.hip), generated at build time.
#include "lane_kernel_src.inc"

namespace {

thread_local std::string g_err;

bpdc_status fail(bpdc_status st, const char* fmt, ...) {
  char buf[1024];
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
    if (e_ != hipSuccess) return fail(BPDC_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

bool csr_ok(const bpdc_csr* A, std::string* why) {
  if (!A || !A->row_ptr || (A->row_ptr[A->rows] > 0 && !A->col_idx)) {
    *why = "null CSR pointer";
    return false;
  }
  if (A->rows < 0 || A->cols < 0) {
    *why = "negative CSR shape";
    return false;
  }
  if (A->row_ptr[0] != 0) {
    *why = "row_ptr[0] != 0";
    return false;
  }
  for (int r = 0; r < A->rows; ++r) {
    if (A->row_ptr[r + 1] < A->row_ptr[r]) {
      *why = "row_ptr not non-decreasing";
      return false;
    }
    for (int k = A->row_ptr[r]; k < A->row_ptr[r + 1]; ++k) {
      const int c = A->col_idx[k];
      if (c < 0 || c >= A->cols) {
        *why = "column index out of range";
        return false;
      }
      if (k > A->row_ptr[r] && c <= A->col_idx[k - 1]) {
        *why = "column indices not sorted and unique within a row";
        return false;
      }
    }
  }
  return true;
}

template <class T>
hipError_t upload(T** dst, const std::vector<T>& src) {
  *dst = nullptr;
  const size_t bytes = std::max<size_t>(1, src.size()) * sizeof(T);
  hipError_t e = hipMalloc((void**)dst, bytes);
  if (e != hipSuccess) return e;
  if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

std::string lib_dir() {
  Dl_info info;
  if (dladdr((void*)&bpdc_version, &info) && info.dli_fname) {
    std::string p = info.dli_fname;
    const size_t k = p.rfind('/');
    if (k != std::string::npos) return p.substr(0, k);
  }
  return ".";
}

std::string cache_dir() {
  const char* env = getenv("BPDC_CACHE_DIR");
  std::string d = env && *env ? std::string(env) : lib_dir() + "/kcache";
  mkdir(d.c_str(), 0755);
  return d;
}

uint64_t fnv1a(const std::string& s, uint64_t h = 1469598103934665603ull) {
  for (unsigned char ch : s) {
    h ^= ch;
    h *= 1099511628211ull;
  }
  return h;
}

const char* kRtcOpts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
const int kNumRtcOpts = sizeof(kRtcOpts) / sizeof(kRtcOpts[0]);

// hipRTC loaded from the ROCm installation by full path instead of linked:
// a process that loaded another copy of hipRTC / comgr first (frameworks ship
// their own) would otherwise compile the lane kernel with that compiler, and
// its code for gfx950 is not the same.
struct Rtc {
  bool ok = false;
  std::string why;
  hiprtcResult (*create)(hiprtcProgram*, const char*, const char*, int, const char**, const char**) = nullptr;
  hiprtcResult (*compile)(hiprtcProgram, int, const char**) = nullptr;
  hiprtcResult (*log_size)(hiprtcProgram, size_t*) = nullptr;
  hiprtcResult (*log)(hiprtcProgram, char*) = nullptr;
  hiprtcResult (*code_size)(hiprtcProgram, size_t*) = nullptr;
  hiprtcResult (*code)(hiprtcProgram, char*) = nullptr;
  hiprtcResult (*destroy)(hiprtcProgram*) = nullptr;
};

const Rtc& rtc() {
  static const Rtc r = [] {
    Rtc x;
    std::vector<std::string> cand;
    if (const char* e = getenv("ROCM_PATH"))
      if (*e) cand.push_back(std::string(e) + "/lib/libhiprtc.so");
    cand.push_back("/opt/rocm/lib/libhiprtc.so");
    // a namespace of its own, so that hipRTC resolves comgr (and everything
    // else) from the installation and not from libraries already loaded
    void* h = nullptr;
    for (auto& c : cand)
      if ((h = dlmopen(LM_ID_NEWLM, c.c_str(), RTLD_NOW | RTLD_LOCAL)) != nullptr) break;
    if (!h) {
      x.why = "libhiprtc.so not found under $ROCM_PATH/lib or /opt/rocm/lib";
      return x;
    }
    x.create = (decltype(x.create))dlsym(h, "hiprtcCreateProgram");
    x.compile = (decltype(x.compile))dlsym(h, "hiprtcCompileProgram");
    x.log_size = (decltype(x.log_size))dlsym(h, "hiprtcGetProgramLogSize");
    x.log = (decltype(x.log))dlsym(h, "hiprtcGetProgramLog");
    x.code_size = (decltype(x.code_size))dlsym(h, "hiprtcGetCodeSize");
    x.code = (decltype(x.code))dlsym(h, "hiprtcGetCode");
    x.destroy = (decltype(x.destroy))dlsym(h, "hiprtcDestroyProgram");
    x.ok = x.create && x.compile && x.log_size && x.log && x.code_size && x.code && x.destroy;
    if (!x.ok) x.why = "libhiprtc.so lacks an expected entry point";
    return x;
  }();
  return r;
}

// Compile (or load from the disk cache) the lane kernel for one code, with
// `chunk` the largest number of shots a wave claims at once (the LDS staging
// of their syndrome words).
bpdc_status lane_code_object(const std::string& spec, int chunk, std::vector<char>* image, std::string* path_out) {
  std::string opts;
  for (int i = 0; i < kNumRtcOpts; ++i) opts += std::string(kRtcOpts[i]) + " ";
  std::string tune;
  if (const char* w = getenv("BPDC_LANE_WPE")) tune += "#define NB_WAVES_PER_EU " + std::string(w) + "\n";
  tune += "#define NB_CHUNK " + std::to_string(chunk) + "\n";
  const std::string full = "using u32 = unsigned int;\n" + std::string(kLaneDeviceSrc) + "\n" + tune + spec + "\n" +
                           std::string(kLaneKernelSrc);
  char key[32];
  snprintf(key, sizeof(key), "%016llx", (unsigned long long)fnv1a(opts + full));
  const std::string path = cache_dir() + "/lane_" + key + ".co";
  if (const char* dump = getenv("BPDC_DUMP_LANE_SOURCE")) {  // for inspecting the generated kernel
    std::ofstream f(std::string(dump) + "/lane_" + key + ".hip");
    f << full;
  }
  if (path_out) *path_out = path;
  {
    std::ifstream f(path, std::ios::binary);
    if (f) {
      image->assign(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
      if (!image->empty()) return BPDC_OK;
    }
  }
  const Rtc& R = rtc();
  if (!R.ok) return fail(BPDC_ERR_UNSUPPORTED, "cannot compile the lane kernel: %s", R.why.c_str());
  hiprtcProgram prog;
  if (R.create(&prog, full.c_str(), "bpdc_lane.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
    return fail(BPDC_ERR_HIP, "hiprtcCreateProgram failed");
  const hiprtcResult rc = R.compile(prog, kNumRtcOpts, kRtcOpts);
  if (rc != HIPRTC_SUCCESS) {
    size_t ls = 0;
    R.log_size(prog, &ls);
    std::string log(ls, '\0');
    if (ls) R.log(prog, &log[0]);
    R.destroy(&prog);
    return fail(BPDC_ERR_HIP, "hipRTC compile of the lane kernel failed: %s", log.substr(0, 800).c_str());
  }
  size_t cs = 0;
  R.code_size(prog, &cs);
  image->resize(cs);
  R.code(prog, image->data());
  R.destroy(&prog);
  const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
  {
    std::ofstream f(tmp, std::ios::binary);
    f.write(image->data(), (std::streamsize)image->size());
  }
  rename(tmp.c_str(), path.c_str());
  return BPDC_OK;
}

}  // namespace

// ------------------------------------------------------------------------------------------
// handles

struct bpdc_code_s {
  bpdc::HostGraph g;
  std::vector<float> lam;
  bpdc::DevCode dev;
  int device = 0;
};

struct LaneKernel {
  hipModule_t mod = nullptr;
  hipFunction_t fn = nullptr;
  hipFunction_t prep = nullptr;  // syndrome preparation kernel of the same module
  int grid = 0;
  int lanes = 1;                 // lanes per shot (64 / lanes shots per one-wave workgroup)
  int spw = 1;                   // prepared syndrome words per lane
  int chunk = 16;                // largest claim of shots (LDS staging)
  std::string cache_path;
};

// One candidate the autotuner timed: what, and ms per 1000 synthetic shots.
struct TuneTry {
  std::string what;
  double ms_per_kshot = -1.0;
};

struct CodePlan {
  int kernel = BPDC_KERNEL_PLAIN;
  LaneKernel lane;
  bpdc::GroupTile tile;
  std::vector<TuneTry> tried;   // the autotuner's measurements (empty when it did not run)
  std::string chose;
};

struct bpdc_plan_s {
  std::vector<bpdc_code> codes;
  bpdc_params params;
  bpdc::KParams kp;
  std::vector<CodePlan> per_code;
  int device = 0;
  int num_cu = 0;
  int max_lds = 0;
  // device table of code descriptors (group kernel, multi-code launch)
  void* d_code_table = nullptr;
  int32_t* d_code_by_rank = nullptr;  // codes by descending column count
  bool multi_ok = false;
  std::string multi_why;
  bpdc::GroupTile multi_tile;
  std::vector<TuneTry> multi_tried;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  uint64_t* dcstats = nullptr;  // DC diagnostics buffer (bpdc_plan_set_dc_stats) or null
  int64_t dcstats_words = 0;
};

namespace {

// Mirrors LaneArgs in lane_kernel.hip.
struct LaneArgsHost {
  const unsigned* synp;
  long long B;
  long long shot_offset;
  unsigned long long* corr;
  unsigned char* flags;
  float* post;
  unsigned long long* cut;
  short* iters;
  const float* lam;
  const int* d_row_ptr;
  const int* d_col;
  unsigned long long* queue;
  float alpha;
  float lsat;
  float tie_eps;
  float lam_uniform;
  int T1;
  int T2;
  int stop;
  int tie_lowest;
  unsigned long long seed;
  float a1_init;
  float a2_init1;
  int skip0;
  unsigned long long* dcstats;
  int soft_period;
  float soft_shift;
};

// Largest lane group the lane kernel may use for one shot (1, 2 or 4).
int lane_max_lanes() {
  const char* e = getenv("BPDC_LANE_MAX_LANES");
  const int v = e ? atoi(e) : 4;
  return v >= 4 ? 4 : (v >= 2 ? 2 : 1);
}

bool uniform_prior(const bpdc_code_s* c) {
  for (float x : c->lam)
    if (x != c->lam[0]) return false;
  return true;
}

bpdc_status build_lane(bpdc_code c, bool posterior, int rule, bool soft, int num_cu, int max_lanes, int chunk,
                       LaneKernel* lk) {
  std::string why;
  if (!bpdc::lane_eligible(c->g, posterior, max_lanes, rule, soft, &why))
    return fail(BPDC_ERR_UNSUPPORTED, "lane kernel cannot run this code: %s", why.c_str());
  std::vector<char> image;
  const bpdc::LaneSpec spec = bpdc::lane_spec(c->g, posterior, uniform_prior(c), max_lanes, rule, soft);
  std::string src = spec.src;
  bpdc_status st = lane_code_object(src, chunk, &image, &lk->cache_path);
  if (st != BPDC_OK) return st;
  lk->lanes = spec.lanes;
  lk->spw = spec.spw;
  lk->chunk = chunk;
  HIP_TRY(hipModuleLoadData(&lk->mod, image.data()));
  HIP_TRY(hipModuleGetFunction(&lk->fn, lk->mod, "bpdc_lane_kernel"));
  HIP_TRY(hipModuleGetFunction(&lk->prep, lk->mod, "bpdc_lane_prepare"));
  int nb = 0;
  HIP_TRY(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lk->fn, 64, 0));
  if (nb < 1) return fail(BPDC_ERR_UNSUPPORTED, "lane kernel does not fit on a compute unit");
  lk->grid = nb * num_cu;
  return BPDC_OK;
}

const size_t kLaneWs = 256;

// queue counter, then the prepared syndrome words [B][lanes][spw]
size_t lane_ws_bytes(const LaneKernel& lk, int64_t B) {
  return kLaneWs + (((size_t)B * lk.lanes * lk.spw * 4 + 255) & ~(size_t)255);
}

bpdc_status lane_launch(const bpdc_plan_s* p, const CodePlan& cp, bpdc_code c, const bpdc::DecodeIO& io,
                        void* ws, hipStream_t stream) {
  unsigned long long* queue = (unsigned long long*)ws;
  (void)hipGetLastError();
  HIP_TRY(bpdc::fill_u64((uint64_t*)queue, 0, 1, stream));
  unsigned* synp = (unsigned*)((char*)ws + kLaneWs);
  {
    const long long B = io.B;
    const unsigned long long* syn = (const unsigned long long*)io.syn;
    void* pargs[] = {&syn, (void*)&B, &synp};
    HIP_TRY(hipModuleLaunchKernel(cp.lane.prep, (unsigned)((io.B + 255) / 256), 1, 1, 256, 1, 1, 0, stream, pargs,
                                  nullptr));
  }
  LaneArgsHost a;
  a.synp = synp;
  a.B = io.B;
  a.shot_offset = io.shot_offset;
  a.corr = (unsigned long long*)io.corr;
  a.flags = io.flags;
  a.post = io.post;
  a.cut = (unsigned long long*)io.cut;
  a.iters = io.iters;
  a.lam = c->dev.lam;
  a.d_row_ptr = c->dev.d_row_ptr;
  a.d_col = c->dev.d_col;
  a.queue = queue;
  a.dcstats = (unsigned long long*)io.dcstats;
  a.soft_period = p->kp.soft_period;
  a.soft_shift = p->kp.soft_shift;
  a.alpha = p->kp.alpha;
  a.lsat = p->kp.lsat;
  a.tie_eps = p->kp.tie_eps;
  a.lam_uniform = c->lam[0];
  a.T1 = p->kp.T1;
  a.T2 = p->kp.T2;
  a.stop = p->kp.stop;
  a.tie_lowest = p->kp.tie_lowest;
  a.seed = p->kp.seed;
  // equal positive priors below the saturation level: the first iteration's
  // check state is the same for every shot up to the syndrome signs
  const float lam0 = c->lam[0];
  a.skip0 = (p->kp.rule == 0 && uniform_prior(c) && lam0 > 0.0f && lam0 < p->kp.lsat && p->kp.T1 >= 1) ? 1 : 0;
  a.a1_init = p->kp.alpha * lam0;
  a.a2_init1 = p->kp.alpha * p->kp.lsat;
  void* args[] = {&a};
  const int64_t want = (io.B * cp.lane.lanes + 63) / 64;
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(cp.lane.grid, want));
  HIP_TRY(hipModuleLaunchKernel(cp.lane.fn, grid, 1, 1, 64, 1, 1, 0, stream, args, nullptr));
  return BPDC_OK;
}

// ---- group kernel: tile selection ---------------------------------------------------------

// Whether the group kernel keeps a per-shot prior array in LDS (the
// posterior second pass, or soft DC in the first pass).
bool group_prior_array(const bpdc_plan_s* p) { return p->kp.second_pass_posterior != 0 || p->kp.soft_period > 0; }

// Sign-bit width of the group kernel's per-check record: 4 bytes for rows of
// at most 32 edges, 8 for longer rows.
int code_info_bytes(const bpdc::DevCode& d) { return d.max_row_deg <= 32 ? 4 : 8; }

// The group kernel variant of a code under a plan: 4 or 8 (min-sum check
// records), 0 (product-sum, per-edge messages).
int group_variant(const bpdc_plan_s* p, const bpdc::DevCode& d) {
  return p->kp.rule == BPDC_RULE_PRODUCT_SUM ? 0 : code_info_bytes(d);
}

bool group_fits(const bpdc_plan_s* p, const bpdc::DevCode& d, std::string* why) {
  if (d.max_row_deg > 58) {
    *why = "row degree above 58";
    return false;
  }
  if (p->kp.rule == BPDC_RULE_PRODUCT_SUM && d.max_row_deg > 8) {
    *why = "product-sum rows above 8 edges";
    return false;
  }
  const size_t lds = bpdc::group_lds_bytes_nm(d.n, d.m, group_prior_array(p), group_variant(p, d), d.E);
  if (lds > (size_t)p->max_lds) {
    *why = "per-shot state of " + std::to_string(lds) + " bytes exceeds the LDS of one workgroup";
    return false;
  }
  return true;
}

// Synthetic shots drawn from the code's own priors (SplitMix64-driven Bernoulli
// errors, s = H e), used only to time candidate launch shapes.
std::vector<uint64_t> autotune_syndromes(const bpdc_code_s* c, int S, uint64_t seed) {
  const int m = c->g.m, n = c->g.n, sw = (m + 63) / 64;
  std::vector<uint64_t> syn((size_t)S * sw, 0);
  std::vector<double> p(n);
  for (int v = 0; v < n; ++v) p[v] = 1.0 / (1.0 + std::exp((double)c->lam[v]));
  uint64_t x = seed;
  for (int b = 0; b < S; ++b) {
    for (int v = 0; v < n; ++v) {
      x += 0x9E3779B97F4A7C15ull;
      uint64_t z = x;
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
      z ^= z >> 31;
      if ((double)(z >> 11) * (1.0 / 9007199254740992.0) < p[v])
        for (int r : c->g.cols[v]) syn[(size_t)b * sw + (r >> 6)] ^= 1ull << (r & 63);
    }
  }
  return syn;
}

struct TuneBuffers {
  uint64_t* syn = nullptr;
  uint64_t* corr = nullptr;
  uint8_t* flags = nullptr;
  unsigned long long* queue = nullptr;
  ~TuneBuffers() {
    if (syn) (void)hipFree(syn);
    if (corr) (void)hipFree(corr);
    if (flags) (void)hipFree(flags);
    if (queue) (void)hipFree(queue);
  }
};

// Time one decode of the synthetic batch with the given group tile (ms), or a
// negative value if it cannot run.  fixed: every shot runs the same number
// of iterations per pass (no early stop, at most 16), the batch that ranks
// thread counts: with the plan's own iteration limits the few shots of a
// short batch that need DC and up to T1 + T2 iterations make the time the
// latency of one shot instead of the throughput being tuned (such a batch of
// the phenomenological DEM ranked 512 threads above 1024, which decode the
// full workload faster).
float time_group(const bpdc_plan_s* p, int code, const bpdc::GroupTile& tile, TuneBuffers& tb, int S, bool fixed) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0f;
  const char* tab = (const char*)p->d_code_table + (size_t)code * sizeof(bpdc::GCodeHost);
  bpdc::KParams kt = p->kp;
  if (fixed) {
    kt.stop = 0;
    kt.T1 = std::min(kt.T1, 16);
    kt.T2 = std::min(kt.T2, 16);
  }
  float best = -1.0f;
  for (int rep = 0; rep < 2; ++rep) {
    (void)hipEventRecord(e0, 0);
    hipError_t e = bpdc::group_launch(tab, nullptr, nullptr, nullptr, kt, tb.syn, nullptr, tb.corr, nullptr, tb.flags,
                                      nullptr, nullptr, nullptr, S, 0, tile.threads, tile.grid, tile.lds_bytes,
                                      tile.info_bytes, tb.queue, 0, nullptr, p->codes[code]->g.n);
    (void)hipEventRecord(e1, 0);
    if (e != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      best = -1.0f;
      break;
    }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (rep == 1) best = ms;  // the first run warms caches and code
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

bpdc_status choose_group_tile(bpdc_plan_s* p, int code, bool autotune, bpdc::GroupTile* out,
                              float* best_ms_out, std::vector<TuneTry>* tried = nullptr,
                              double* best_ms_per_kshot = nullptr) {
  const bpdc::DevCode& d = p->codes[code]->dev;
  bpdc::GroupTile base;
  base.info_bytes = group_variant(p, d);
  base.lds_bytes = bpdc::group_lds_bytes_nm(d.n, d.m, group_prior_array(p), base.info_bytes, d.E);
  // powers of two (thread counts that split a phase into whole rounds, such
  // as 896 for 2592 checks, measured slower than 1024 on every code tried:
  // fewer waves hide less latency)
  std::vector<int> cands;
  const int work = std::max(d.n, d.m);
  for (int t : {64, 128, 256, 512, 1024}) {
    if (t > 64 && t / 2 >= work) continue;  // more threads than items
    cands.push_back(t);
  }
  if (const char* e = getenv("BPDC_GROUP_THREADS"))  // pins the threads per workgroup
    cands = {std::min(1024, std::max(64, atoi(e) / 64 * 64))};
  auto make = [&](int threads) {
    bpdc::GroupTile t = base;
    t.threads = threads;
    const int nb = bpdc::group_occupancy(threads, t.lds_bytes, t.info_bytes, p->max_lds);
    t.grid = std::max(1, nb) * p->num_cu;
    return t;
  };
  if (!autotune) {
    int th = 64;
    while (th < 512 && th < std::max(d.m, d.n / 2)) th *= 2;
    *out = make(th);
    if (best_ms_out) *best_ms_out = -1.0f;
    return BPDC_OK;
  }
  // enough shots to fill every workgroup slot twice (throughput, not the
  // latency of a few shots), more for small codes
  const int S = (int)std::max<int64_t>(4 * p->num_cu, std::min<int64_t>(4096, (1 << 21) / std::max(1, d.E)));
  TuneBuffers tb;
  const int sw = (d.m + 63) / 64, nw = (d.n + 63) / 64;
  std::vector<uint64_t> hs = autotune_syndromes(p->codes[code], S, 0x5EED0000ull + (uint64_t)code);
  HIP_TRY(hipMalloc((void**)&tb.syn, hs.size() * 8));
  HIP_TRY(hipMemcpy(tb.syn, hs.data(), hs.size() * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMalloc((void**)&tb.corr, (size_t)S * nw * 8));
  HIP_TRY(hipMalloc((void**)&tb.flags, (size_t)S));
  HIP_TRY(hipMalloc((void**)&tb.queue, 256));
  (void)sw;
  float best = -1.0f;
  for (int th : cands) {
    bpdc::GroupTile t = make(th);
    if (bpdc::group_occupancy(th, t.lds_bytes, t.info_bytes, p->max_lds) < 1) continue;
    const float ms = time_group(p, code, t, tb, S, true);
    if (tried) {
      TuneTry tt;
      tt.what = "group " + std::to_string(th) + " threads, 1 shot/workgroup, " + std::to_string(t.lds_bytes) +
                " B LDS per shot, " + std::to_string(t.grid / p->num_cu) +
                " workgroups/CU (16 + 16 iterations, no early stop)";
      tt.ms_per_kshot = ms > 0 ? ms * 1000.0 / S : -1.0;
      tried->push_back(tt);
    }
    if (ms > 0 && (best < 0 || ms < best)) {
      best = ms;
      *out = t;
    }
  }
  if (best < 0)
    return fail(BPDC_ERR_UNSUPPORTED, "no group tile could run code %d (lds %zu of %d bytes, last HIP error: %s)",
                code, base.lds_bytes, p->max_lds, hipGetErrorString(hipGetLastError()));
  if (best_ms_per_kshot) {
    // the chosen tile on the same batch with the plan's own iterations: the
    // figure AUTO compares with the lane kernel's
    const float ms = time_group(p, code, *out, tb, S, false);
    *best_ms_per_kshot = ms > 0 ? ms * 1000.0 / S : -1.0;
    if (tried) {
      TuneTry tt;
      tt.what = "group " + std::to_string(out->threads) + " threads as chosen, the plan's iterations";
      tt.ms_per_kshot = *best_ms_per_kshot;
      tried->push_back(tt);
    }
  }
  if (best_ms_out) *best_ms_out = best;
  return BPDC_OK;
}

// ---- lane kernel: tile selection ----------------------------------------------------------

// Lane-tile candidates of a code: the lane-group sizes its symmetry allows
// (the largest, halved down to one lane per shot: 64, 32 or 16 shots per
// one-wave workgroup) and the largest claim of shots (LDS staging of their
// syndrome words).  BPDC_LANE_CHUNK pins the claim size.
std::vector<std::pair<int, int>> lane_candidates(const bpdc::HostGraph& g, bool posterior, bool uniform, int rule,
                                                 bool soft) {
  std::vector<int> lanes;
  for (int L = lane_max_lanes(); L >= 1; L /= 2) {
    std::string why;
    if (!bpdc::lane_eligible(g, posterior, L, rule, soft, &why)) continue;
    const int got = bpdc::lane_spec(g, posterior, uniform, L, rule, soft).lanes;
    if (std::find(lanes.begin(), lanes.end(), got) == lanes.end()) lanes.push_back(got);
  }
  std::vector<int> chunks = {8, 16, 32};
  if (const char* e = getenv("BPDC_LANE_CHUNK")) chunks = {std::max(1, atoi(e))};
  std::vector<std::pair<int, int>> out;
  for (int L : lanes)
    for (int ch : chunks) out.push_back({L, ch});
  // the default tile (largest lane group, claims of 16) first: the tuner keeps it
  // unless another is faster by more than the timing noise
  std::stable_sort(out.begin(), out.end(), [&](const std::pair<int, int>& a, const std::pair<int, int>& b) {
    return (a.first == lanes[0] && a.second == 16) > (b.first == lanes[0] && b.second == 16);
  });
  return out;
}

struct LaneTuneBuffers {
  uint64_t* syn = nullptr;
  uint64_t* corr = nullptr;
  uint8_t* flags = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  ~LaneTuneBuffers() {
    if (syn) (void)hipFree(syn);
    if (corr) (void)hipFree(corr);
    if (flags) (void)hipFree(flags);
    if (ws) (void)hipFree(ws);
  }
};

// Time one decode of S synthetic shots with a lane tile (ms), negative if it fails.
float time_lane(const bpdc_plan_s* p, const CodePlan& cp, bpdc_code c, LaneTuneBuffers& tb, int64_t S) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0f;
  bpdc::DecodeIO io{tb.syn, S, 0, tb.corr, tb.flags, nullptr, nullptr, nullptr, nullptr};
  float best = -1.0f;
  for (int rep = 0; rep < 2; ++rep) {
    (void)hipEventRecord(e0, 0);
    const bpdc_status st = lane_launch(p, cp, c, io, tb.ws, 0);
    (void)hipEventRecord(e1, 0);
    if (st != BPDC_OK || hipEventSynchronize(e1) != hipSuccess) {
      best = -1.0f;
      break;
    }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (rep == 1) best = ms;  // the first run warms caches and code
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

// Build the lane kernel of code `code` into cp.lane: with `autotune`, every
// candidate tile is compiled (or found in the kernel cache) and timed on
// synthetic shots drawn from the code's priors, and the fastest is kept;
// otherwise the largest lane group with claims of 16.  *best_ms_per_kshot
// gets the kept tile's time per 1000 shots (negative when not timed).
bpdc_status choose_lane(bpdc_plan_s* p, int code, bool autotune, CodePlan* cp, double* best_ms_per_kshot) {
  bpdc_code c = p->codes[code];
  const bool posterior = p->kp.second_pass_posterior != 0, soft = p->kp.soft_period > 0;
  const int rule = p->kp.rule;
  if (best_ms_per_kshot) *best_ms_per_kshot = -1.0;
  std::vector<std::pair<int, int>> cands = lane_candidates(c->g, posterior, uniform_prior(c), rule, soft);
  if (cands.empty()) {
    std::string why;
    bpdc::lane_eligible(c->g, posterior, lane_max_lanes(), rule, soft, &why);
    return fail(BPDC_ERR_UNSUPPORTED, "lane kernel cannot run code %d: %s", code, why.c_str());
  }
  if (!autotune || cands.size() == 1) {
    const int ch = getenv("BPDC_LANE_CHUNK") ? cands[0].second : 16;
    return build_lane(c, posterior, rule, soft, p->num_cu, cands[0].first, ch, &cp->lane);
  }
  // enough shots for several rounds of the persistent grid (steady state, not the
  // end of the batch), at most 64 MB of syndromes and corrections
  const int sw = (c->g.m + 63) / 64, nw = (c->g.n + 63) / 64;
  const int64_t S = std::max<int64_t>(8192, std::min<int64_t>(262144, (64ll << 20) / (8 * (sw + nw))));
  LaneTuneBuffers tb;
  const std::vector<uint64_t> hs = autotune_syndromes(c, (int)S, 0x1A4E0000ull + (uint64_t)code);
  HIP_TRY(hipMalloc((void**)&tb.syn, hs.size() * 8));
  HIP_TRY(hipMemcpy(tb.syn, hs.data(), hs.size() * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMalloc((void**)&tb.corr, (size_t)S * nw * 8));
  HIP_TRY(hipMalloc((void**)&tb.flags, (size_t)S));
  (void)sw;
  double best = -1.0;
  cp->tried.clear();
  for (const auto& cand : cands) {
    CodePlan trial;
    bpdc_status st = build_lane(c, posterior, rule, soft, p->num_cu, cand.first, cand.second, &trial.lane);
    if (st != BPDC_OK) {
      if (trial.lane.mod) (void)hipModuleUnload(trial.lane.mod);
      continue;
    }
    const size_t need = lane_ws_bytes(trial.lane, S);
    if (need > tb.ws_bytes) {
      if (tb.ws) (void)hipFree(tb.ws);
      tb.ws = nullptr;
      HIP_TRY(hipMalloc(&tb.ws, need));
      tb.ws_bytes = need;
    }
    trial.kernel = BPDC_KERNEL_LANE;
    const float ms = time_lane(p, trial, c, tb, S);
    TuneTry t;
    t.what = "lane " + std::to_string(trial.lane.lanes) + " lanes/shot, " + std::to_string(64 / trial.lane.lanes) +
             " shots/workgroup, claims of " + std::to_string(trial.lane.chunk);
    t.ms_per_kshot = ms > 0 ? ms * 1000.0 / (double)S : -1.0;
    cp->tried.push_back(t);
    // a candidate replaces the one kept only when it is faster by more than 1 %
    // (repeated timings of one tile differ by about that much)
    if (ms > 0 && (best < 0 || t.ms_per_kshot < 0.99 * best)) {
      best = t.ms_per_kshot;
      if (cp->lane.mod) (void)hipModuleUnload(cp->lane.mod);
      cp->lane = trial.lane;
    } else if (trial.lane.mod) {
      (void)hipModuleUnload(trial.lane.mod);
    }
  }
  if (best < 0) return fail(BPDC_ERR_UNSUPPORTED, "no lane tile could run code %d", code);
  if (best_ms_per_kshot) *best_ms_per_kshot = best;
  return BPDC_OK;
}

bpdc_status build_code_table(bpdc_plan_s* p) {
  std::vector<bpdc::GCodeHost> tab(p->codes.size());
  std::vector<int32_t> rank(p->codes.size());
  for (size_t i = 0; i < p->codes.size(); ++i) {
    const bpdc::DevCode& d = p->codes[i]->dev;
    tab[i] = {d.n, d.m, d.md, p->kp.second_pass_posterior, d.h_row_ptr, d.h_col, d.h_col_ptr, d.h_col_edge,
              d.h_edge_row, d.d_row_ptr, d.d_col, d.lam, d.v_ell, d.c_ell, d.v_blk_deg, d.max_col_deg, d.max_row_deg,
              d.g_lam, d.g_dcol, d.g_pos};
    rank[i] = (int32_t)i;
  }
  std::stable_sort(rank.begin(), rank.end(),
                   [&](int a, int b) { return p->codes[a]->dev.n > p->codes[b]->dev.n; });
  HIP_TRY(hipMalloc(&p->d_code_table, tab.size() * sizeof(bpdc::GCodeHost)));
  HIP_TRY(hipMemcpy(p->d_code_table, tab.data(), tab.size() * sizeof(bpdc::GCodeHost), hipMemcpyHostToDevice));
  HIP_TRY(hipMalloc((void**)&p->d_code_by_rank, rank.size() * sizeof(int32_t)));
  HIP_TRY(hipMemcpy(p->d_code_by_rank, rank.data(), rank.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  return BPDC_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Multi-code workspace: the shot counter, the per-code histogram and bases of
// the ordering sort (one extra bucket each for out-of-range code indices), and
// the processing order.
size_t multi_ws_bytes(const bpdc_plan_s* p, int64_t B) {
  return 256 + 2 * align256((p->codes.size() + 1) * 4) + align256((size_t)std::max<int64_t>(B, 1) * 4);
}

bpdc_status multi_enqueue(bpdc_plan_s* p, const int32_t* cos, const uint64_t* syn, const int64_t* syn_off,
                          uint64_t* corr, const int64_t* corr_off, uint8_t* flags, int16_t* iters, int64_t B,
                          int64_t shot_offset, void* ws, hipStream_t s, const bpdc::GroupTile* tile = nullptr,
                          unsigned long long* dcstats = nullptr, const bpdc::KParams* kp = nullptr) {
  const bpdc::GroupTile& t = tile ? *tile : p->multi_tile;
  char* w = (char*)ws;
  unsigned long long* queue = (unsigned long long*)w;
  unsigned* hist = (unsigned*)(w + 256);
  unsigned* base = (unsigned*)(w + 256 + align256((p->codes.size() + 1) * 4));
  int32_t* order = (int32_t*)(w + 256 + 2 * align256((p->codes.size() + 1) * 4));
  HIP_TRY(bpdc::group_order(cos, B, p->d_code_by_rank, (int)p->codes.size(), hist, base, order, flags, s));
  HIP_TRY(bpdc::group_launch(p->d_code_table, hist + p->codes.size(), cos, order, kp ? *kp : p->kp, syn, syn_off, corr,
                             corr_off, flags, nullptr,
                             nullptr, iters, B, shot_offset, t.threads, t.grid, t.lds_bytes, t.info_bytes, queue, s,
                             dcstats));
  return BPDC_OK;
}

// Threads per workgroup of the multi-code launch: each candidate is timed on a
// synthetic mixed batch (32 shots of every code drawn from its priors, codes
// interleaved; every shot runs min(16, T) iterations per pass without early
// stop, as for a single code's group tile) and the fastest kept.  The LDS per
// workgroup is the largest code's state either way.
bpdc_status choose_multi_tile(bpdc_plan_s* p, const bpdc::GroupTile& base, const std::vector<int>& cands) {
  const int nc = (int)p->codes.size();
  const int per = 32;
  const int64_t B = (int64_t)nc * per;
  std::vector<std::vector<uint64_t>> syn_c(nc);
  for (int i = 0; i < nc; ++i) syn_c[i] = autotune_syndromes(p->codes[i], per, 0x3C0D0000ull + (uint64_t)i);
  std::vector<int32_t> cos((size_t)B);
  std::vector<int64_t> so((size_t)B), co((size_t)B);
  std::vector<uint64_t> syn;
  int64_t sw_tot = 0, nw_tot = 0;
  for (int k = 0; k < per; ++k)
    for (int i = 0; i < nc; ++i) {
      const int64_t b = (int64_t)k * nc + i;
      const int sw = (p->codes[i]->g.m + 63) / 64, nw = (p->codes[i]->g.n + 63) / 64;
      cos[b] = i;
      so[b] = sw_tot;
      co[b] = nw_tot;
      syn.insert(syn.end(), syn_c[i].begin() + (size_t)k * sw, syn_c[i].begin() + (size_t)(k + 1) * sw);
      sw_tot += sw;
      nw_tot += nw;
    }
  struct Bufs {
    void* p[7] = {};
    ~Bufs() {
      for (void* x : p)
        if (x) (void)hipFree(x);
    }
  } d;
  const size_t wsb = multi_ws_bytes(p, B);
  HIP_TRY(hipMalloc(&d.p[0], cos.size() * 4));
  HIP_TRY(hipMalloc(&d.p[1], so.size() * 8));
  HIP_TRY(hipMalloc(&d.p[2], co.size() * 8));
  HIP_TRY(hipMalloc(&d.p[3], syn.size() * 8));
  HIP_TRY(hipMalloc(&d.p[4], (size_t)nw_tot * 8));
  HIP_TRY(hipMalloc(&d.p[5], (size_t)B));
  HIP_TRY(hipMalloc(&d.p[6], wsb));
  HIP_TRY(hipMemcpy(d.p[0], cos.data(), cos.size() * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(d.p[1], so.data(), so.size() * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(d.p[2], co.data(), co.size() * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(d.p[3], syn.data(), syn.size() * 8, hipMemcpyHostToDevice));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  bpdc::KParams kt = p->kp;
  kt.stop = 0;
  kt.T1 = std::min(kt.T1, 16);
  kt.T2 = std::min(kt.T2, 16);
  double best = -1.0;
  p->multi_tried.clear();
  for (int th : cands) {
    bpdc::GroupTile t = base;
    t.threads = th;
    const int nb = bpdc::group_occupancy(th, t.lds_bytes, t.info_bytes, p->max_lds);
    if (nb < 1) continue;
    t.grid = nb * p->num_cu;
    float ms = -1.0f;
    for (int rep = 0; rep < 2; ++rep) {
      (void)hipEventRecord(e0, 0);
      const bpdc_status st = multi_enqueue(p, (const int32_t*)d.p[0], (const uint64_t*)d.p[3], (const int64_t*)d.p[1],
                                           (uint64_t*)d.p[4], (const int64_t*)d.p[2], (uint8_t*)d.p[5], nullptr, B, 0,
                                           d.p[6], 0, &t, nullptr, &kt);
      (void)hipEventRecord(e1, 0);
      if (st != BPDC_OK || hipEventSynchronize(e1) != hipSuccess) {
        ms = -1.0f;
        break;
      }
      (void)hipEventElapsedTime(&ms, e0, e1);
    }
    TuneTry tt;
    tt.what = "multi-code " + std::to_string(th) + " threads, " + std::to_string(nb) +
              " workgroups/CU (16 + 16 iterations, no early stop)";
    tt.ms_per_kshot = ms > 0 ? ms * 1000.0 / (double)B : -1.0;
    p->multi_tried.push_back(tt);
    if (ms > 0 && (best < 0 || tt.ms_per_kshot < best)) {
      best = tt.ms_per_kshot;
      p->multi_tile = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipGetLastError();
  if (best < 0) return fail(BPDC_ERR_UNSUPPORTED, "no multi-code tile could run");
  return BPDC_OK;
}

}  // namespace

namespace {
std::string json_str(const std::string& x) {
  std::string o = "\"";
  for (char ch : x) {
    if (ch == '"' || ch == '\\') o += '\\';
    o += ch;
  }
  return o + "\"";
}
std::string json_tried(const std::vector<TuneTry>& v) {
  std::string o = "[";
  for (size_t k = 0; k < v.size(); ++k) {
    char b[64];
    snprintf(b, sizeof(b), "%.5g", v[k].ms_per_kshot);
    o += (k ? ", " : "") + std::string("{\"candidate\": ") + json_str(v[k].what) + ", \"ms_per_1000_shots\": " + b + "}";
  }
  return o + "]";
}
}  // namespace

extern "C" {

const char* bpdc_version(void) { return "bpdc 0.1 gfx950 (plain, lane[hipRTC], group)"; }

const char* bpdc_status_string(bpdc_status s) {
  switch (s) {
    case BPDC_OK: return "ok";
    case BPDC_ERR_INVALID_ARG: return "invalid argument";
    case BPDC_ERR_UNSUPPORTED: return "unsupported";
    case BPDC_ERR_WORKSPACE: return "workspace too small";
    case BPDC_ERR_HIP: return "HIP runtime error";
    case BPDC_ERR_OOM: return "out of device memory";
    default: return "unknown status";
  }
}

const char* bpdc_last_error(void) { return g_err.c_str(); }

bpdc_status bpdc_code_create(const bpdc_csr* H, const bpdc_csr* D, const double* h_priors, bpdc_code* out) {
  if (!out) return fail(BPDC_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  if (!H || !D || !h_priors) return fail(BPDC_ERR_INVALID_ARG, "null H, D or priors");
  std::string why;
  if (!csr_ok(H, &why)) return fail(BPDC_ERR_INVALID_ARG, "H: %s", why.c_str());
  if (!csr_ok(D, &why)) return fail(BPDC_ERR_INVALID_ARG, "D: %s", why.c_str());
  if (D->cols != H->cols) return fail(BPDC_ERR_INVALID_ARG, "D has %d columns, H has %d", D->cols, H->cols);
  if (H->cols < 1 || H->rows < 1) return fail(BPDC_ERR_INVALID_ARG, "empty H");
  for (int v = 0; v < H->cols; ++v)
    if (!(h_priors[v] > 0.0 && h_priors[v] < 1.0))
      return fail(BPDC_ERR_INVALID_ARG, "prior %d = %g outside (0, 1)", v, h_priors[v]);
  auto c = std::make_unique<bpdc_code_s>();
  bpdc::HostGraph& g = c->g;
  g.n = H->cols;
  g.m = H->rows;
  g.rows.resize(g.m);
  g.cols.resize(g.n);
  for (int r = 0; r < g.m; ++r)
    for (int k = H->row_ptr[r]; k < H->row_ptr[r + 1]; ++k) {
      g.rows[r].push_back(H->col_idx[k]);
      g.cols[H->col_idx[k]].push_back(r);
    }
  g.drows.resize(D->rows);
  for (int r = 0; r < D->rows; ++r)
    for (int k = D->row_ptr[r]; k < D->row_ptr[r + 1]; ++k) g.drows[r].push_back(D->col_idx[k]);
  bpdc::DevCode& d = c->dev;
  d.n = g.n;
  d.m = g.m;
  d.md = D->rows;
  d.E = H->row_ptr[H->rows];
  d.dnnz = D->row_ptr[D->rows];
  for (auto& r : g.rows) d.max_row_deg = std::max(d.max_row_deg, (int)r.size());
  for (auto& r : g.cols) d.max_col_deg = std::max(d.max_col_deg, (int)r.size());
  for (auto& r : g.drows) d.max_drow_deg = std::max(d.max_drow_deg, (int)r.size());
  if (d.max_row_deg > 64) return fail(BPDC_ERR_UNSUPPORTED, "H row degree %d above 64", d.max_row_deg);
  if (d.max_col_deg > 16) return fail(BPDC_ERR_UNSUPPORTED, "H column degree %d above 16", d.max_col_deg);
  if (d.max_drow_deg > 32) return fail(BPDC_ERR_UNSUPPORTED, "D row degree %d above 32", d.max_drow_deg);
  // prior LLR: log((1 - p) / p) in double, rounded once to float
  c->lam.resize(g.n);
  for (int v = 0; v < g.n; ++v) c->lam[v] = (float)std::log((1.0 - h_priors[v]) / h_priors[v]);
  // CSR / CSC / D arrays
  std::vector<int32_t> hrp(H->row_ptr, H->row_ptr + g.m + 1), hci(H->col_idx, H->col_idx + d.E);
  std::vector<int32_t> cp(g.n + 1, 0), ce, er(d.E);
  for (int r = 0; r < g.m; ++r)
    for (int k = hrp[r]; k < hrp[r + 1]; ++k) er[k] = r;
  {
    std::vector<std::vector<int32_t>> per(g.n);
    for (int r = 0; r < g.m; ++r)
      for (int k = hrp[r]; k < hrp[r + 1]; ++k) per[hci[k]].push_back(k);
    for (int v = 0; v < g.n; ++v) {
      cp[v + 1] = cp[v] + (int)per[v].size();
      ce.insert(ce.end(), per[v].begin(), per[v].end());
    }
  }
  std::vector<int32_t> drp(D->row_ptr, D->row_ptr + D->rows + 1), dci(D->col_idx, D->col_idx + d.dnnz);
  // The group kernel's min-sum variants keep the posteriors in LDS in slot
  // order.  For codes with rows above 32 edges (the 64-bit-record variant)
  // that is the columns sorted by descending degree (ties in column order),
  // so that a block of 64 slots mostly holds columns of one degree and the
  // variant's per-block degree bound (each wave's variable phase stops at its
  // block's largest degree) wastes little on padding: circuit-level BB144
  // DEM 215 -> 211 ms.  Other codes keep the column order (the 32-bit variant
  // runs every column to the code's largest degree, and the sorted order
  // measured 1-2 % slower there).  g_lam holds the priors and g_dcol the rows
  // of D in slot terms (each row's entries still in ascending column order,
  // the order of DC's tie draw); g_pos maps a column to its slot for the
  // outputs.
  std::vector<int32_t> slot_col(g.n), col_slot(g.n);
  for (int v = 0; v < g.n; ++v) slot_col[v] = v;
  if (code_info_bytes(d) == 8)
    std::stable_sort(slot_col.begin(), slot_col.end(),
                     [&](int a, int b) { return cp[a + 1] - cp[a] > cp[b + 1] - cp[b]; });
  for (int q = 0; q < g.n; ++q) col_slot[slot_col[q]] = q;
  std::vector<float> glam(g.n);
  for (int q = 0; q < g.n; ++q) glam[q] = c->lam[slot_col[q]];
  std::vector<int32_t> gdcol(dci.size());
  for (size_t k = 0; k < dci.size(); ++k) gdcol[k] = col_slot[dci[k]];
  // padded slot-major adjacency for the group kernel (one coalesced load per
  // edge), in the forms its min-sum phases use directly: a slot's entry is
  // ((check + kLdsHead / 16) << 10) | position in the check's row (>> 6: the LDS address
  // of the check's 16-byte record, after kLdsHead bytes of control words), a
  // check's entry the LDS address of its column's posterior (at the column's
  // slot), which follows the m + 1 records.  Padding: check m / slot n,
  // dummies that the group kernel keeps in LDS.  (Codes too large for one
  // workgroup's LDS never run the group kernel; their entries wrap harmlessly
  // in unsigned arithmetic.)
  static_assert(bpdc::kLdsHead % 16 == 0, "check records are 16-byte aligned");
  const uint32_t rec0 = bpdc::kLdsHead / 16, l_off = (uint32_t)bpdc::kLdsHead + ((uint32_t)g.m + 1u) * 16u;
  std::vector<int32_t> vell((size_t)std::max(1, d.max_col_deg) * g.n, (int32_t)(((uint32_t)g.m + rec0) << 10)),
      cell((size_t)std::max(1, d.max_row_deg) * g.m, (int32_t)(l_off + 4u * (uint32_t)g.n));
  for (int v = 0; v < g.n; ++v)
    for (int k = cp[v]; k < cp[v + 1]; ++k) {
      const int edge = ce[k], r = er[edge];
      vell[(size_t)(k - cp[v]) * g.n + col_slot[v]] =
          (int32_t)((((uint32_t)r + rec0) << 10) | (uint32_t)(edge - hrp[r]));
    }
  for (int r = 0; r < g.m; ++r)
    for (int k = hrp[r]; k < hrp[r + 1]; ++k)
      cell[(size_t)(k - hrp[r]) * g.m + r] = (int32_t)(l_off + 4u * (uint32_t)col_slot[hci[k]]);
  std::vector<int32_t> vblk((size_t)std::max(1, (g.n + 63) / 64), 0);
  for (int v = 0; v < g.n; ++v) vblk[col_slot[v] >> 6] = std::max(vblk[col_slot[v] >> 6], cp[v + 1] - cp[v]);
  if (hipGetDevice(&c->device) != hipSuccess) return fail(BPDC_ERR_HIP, "no HIP device");
  hipError_t e;
  if ((e = upload(&d.h_row_ptr, hrp)) != hipSuccess || (e = upload(&d.h_col, hci)) != hipSuccess ||
      (e = upload(&d.h_col_ptr, cp)) != hipSuccess || (e = upload(&d.h_col_edge, ce)) != hipSuccess ||
      (e = upload(&d.h_edge_row, er)) != hipSuccess || (e = upload(&d.d_row_ptr, drp)) != hipSuccess ||
      (e = upload(&d.d_col, dci)) != hipSuccess || (e = upload(&d.lam, c->lam)) != hipSuccess ||
      (e = upload(&d.v_ell, vell)) != hipSuccess || (e = upload(&d.c_ell, cell)) != hipSuccess ||
      (e = upload(&d.v_blk_deg, vblk)) != hipSuccess || (e = upload(&d.g_lam, glam)) != hipSuccess ||
      (e = upload(&d.g_dcol, gdcol)) != hipSuccess || (e = upload(&d.g_pos, col_slot)) != hipSuccess) {
    bpdc_code_destroy(c.release());
    return fail(e == hipErrorOutOfMemory ? BPDC_ERR_OOM : BPDC_ERR_HIP, "upload: %s", hipGetErrorString(e));
  }
  *out = c.release();
  return BPDC_OK;
}

bpdc_status bpdc_code_destroy(bpdc_code c) {
  if (!c) return BPDC_OK;
  bpdc::DevCode& d = c->dev;
  void* ptrs[] = {d.h_row_ptr, d.h_col, d.h_col_ptr, d.h_col_edge, d.h_edge_row, d.d_row_ptr, d.d_col,
                  d.lam,       d.v_ell, d.c_ell,     d.v_blk_deg,  d.g_lam,      d.g_dcol,    d.g_pos};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete c;
  return BPDC_OK;
}

bpdc_status bpdc_code_info(bpdc_code c, int32_t* n, int32_t* m, int32_t* md, int32_t* edges) {
  if (!c) return fail(BPDC_ERR_INVALID_ARG, "null code");
  if (n) *n = c->dev.n;
  if (m) *m = c->dev.m;
  if (md) *md = c->dev.md;
  if (edges) *edges = c->dev.E;
  return BPDC_OK;
}

bpdc_status bpdc_lane_precompile(const bpdc_csr* H, const bpdc_csr* D, int32_t posterior, int32_t uniform_prior,
                                 int32_t rule, int32_t soft) {
  if (rule != BPDC_RULE_MIN_SUM && rule != BPDC_RULE_PRODUCT_SUM) return fail(BPDC_ERR_INVALID_ARG, "bad rule");
  std::string why;
  if (!H || !D || !csr_ok(H, &why) || !csr_ok(D, &why) || H->cols != D->cols)
    return fail(BPDC_ERR_INVALID_ARG, "bad CSR: %s", why.c_str());
  bpdc::HostGraph g;
  g.n = H->cols;
  g.m = H->rows;
  g.rows.resize(g.m);
  g.cols.resize(g.n);
  for (int r = 0; r < g.m; ++r)
    for (int k = H->row_ptr[r]; k < H->row_ptr[r + 1]; ++k) {
      g.rows[r].push_back(H->col_idx[k]);
      g.cols[H->col_idx[k]].push_back(r);
    }
  g.drows.resize(D->rows);
  for (int r = 0; r < D->rows; ++r)
    for (int k = D->row_ptr[r]; k < D->row_ptr[r + 1]; ++k) g.drows[r].push_back(D->col_idx[k]);
  if (!bpdc::lane_eligible(g, posterior != 0, lane_max_lanes(), rule, soft != 0, &why))
    return fail(BPDC_ERR_UNSUPPORTED, "lane kernel cannot run this code: %s", why.c_str());
  // every tile the autotuner may time
  for (const auto& cand : lane_candidates(g, posterior != 0, uniform_prior != 0, rule, soft != 0)) {
    std::vector<char> image;
    const bpdc_status st = lane_code_object(
        bpdc::lane_spec(g, posterior != 0, uniform_prior != 0, cand.first, rule, soft != 0).src, cand.second, &image,
        nullptr);
    if (st != BPDC_OK) return st;
  }
  return BPDC_OK;
}

bpdc_status bpdc_plan_create(const bpdc_code* codes, int32_t ncodes, const bpdc_params* params,
                             int32_t kernel, bpdc_plan* out) {
  if (!out) return fail(BPDC_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  if (!codes || ncodes < 1 || !params) return fail(BPDC_ERR_INVALID_ARG, "need >= 1 code and params");
  for (int i = 0; i < ncodes; ++i)
    if (!codes[i]) return fail(BPDC_ERR_INVALID_ARG, "code %d is null", i);
  const bpdc_params& P = *params;
  if (P.max_iter[0] < 1 || P.max_iter[1] < 1 || P.max_iter[0] > 32767 || P.max_iter[1] > 32767)
    return fail(BPDC_ERR_INVALID_ARG, "max_iter must be in [1, 32767]");
  if (!(P.llr_sat > 0.0f) || !std::isfinite(P.llr_sat)) return fail(BPDC_ERR_INVALID_ARG, "llr_sat must be finite and > 0");
  if (!(P.tie_eps >= 0.0f) || !std::isfinite(P.tie_eps)) return fail(BPDC_ERR_INVALID_ARG, "tie_eps must be >= 0");
  if (!std::isfinite(P.alpha) || !(P.alpha >= 0.0f)) return fail(BPDC_ERR_INVALID_ARG, "alpha must be finite and >= 0");
  if (P.second_pass_prior != BPDC_PRIOR_CHANNEL && P.second_pass_prior != BPDC_PRIOR_POSTERIOR)
    return fail(BPDC_ERR_INVALID_ARG, "bad second_pass_prior");
  if (P.rule != BPDC_RULE_MIN_SUM && P.rule != BPDC_RULE_PRODUCT_SUM)
    return fail(BPDC_ERR_INVALID_ARG, "bad rule");
  if (P.soft_period < 0 || P.soft_period > 32767) return fail(BPDC_ERR_INVALID_ARG, "soft_period must be in [0, 32767]");
  if (P.soft_period > 0 && !(P.soft_shift >= 0.0f && std::isfinite(P.soft_shift)))
    return fail(BPDC_ERR_INVALID_ARG, "soft_shift must be finite and >= 0");
  if (P.rule == BPDC_RULE_PRODUCT_SUM)
    for (int i = 0; i < ncodes; ++i)
      if (codes[i]->dev.max_row_deg > 32)
        return fail(BPDC_ERR_UNSUPPORTED, "product-sum: code %d has a row of degree %d (at most 32)", i,
                    codes[i]->dev.max_row_deg);
  if (P.tie_break != BPDC_TIE_HASH && P.tie_break != BPDC_TIE_LOWEST_INDEX)
    return fail(BPDC_ERR_INVALID_ARG, "bad tie_break");
  if (kernel < BPDC_KERNEL_AUTO || kernel > BPDC_KERNEL_GROUP) return fail(BPDC_ERR_INVALID_ARG, "bad kernel");
  auto p = std::make_unique<bpdc_plan_s>();
  p->codes.assign(codes, codes + ncodes);
  p->params = P;
  p->kp.T1 = P.max_iter[0];
  p->kp.T2 = P.max_iter[1];
  p->kp.alpha = P.alpha + 0.0f;  // -0 becomes +0: every message magnitude is then +0 or positive
  p->kp.lsat = P.llr_sat;
  p->kp.tie_eps = P.tie_eps;
  p->kp.second_pass_posterior = P.second_pass_prior == BPDC_PRIOR_POSTERIOR;
  p->kp.stop = P.stop_on_converge != 0;
  p->kp.tie_lowest = P.tie_break == BPDC_TIE_LOWEST_INDEX;
  p->kp.seed = P.seed;
  p->kp.rule = P.rule;
  p->kp.soft_period = P.soft_period;
  p->kp.soft_shift = P.soft_period > 0 ? P.soft_shift : 0.0f;
  HIP_TRY(hipGetDevice(&p->device));
  {  // set-up of bpdc_decode_noalloc on this device: the static scratch's device address, once per
     // device (a failure is reported by bpdc_decode_noalloc itself, which looks it up again)
    void* scratch = nullptr;
    if (bpdc::noalloc_scratch(p->device, &scratch) != hipSuccess) (void)hipGetLastError();
  }
  // the group kernels read LDS addresses from the code tables, valid only
  // while their dynamic LDS starts at address 0 (no static LDS)
  if (!bpdc::group_lds_starts_at_zero())
    return fail(BPDC_ERR_HIP, "the group kernels were built with static LDS: their code tables do not apply");
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, p->device));
  p->num_cu = prop.multiProcessorCount;
  {
    int optin = 0;
    if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, p->device) != hipSuccess)
      optin = 0;
    p->max_lds = std::max<int>((int)prop.sharedMemPerBlock, optin);
  }
  p->per_code.resize(ncodes);
  bpdc_status st = build_code_table(p.get());
  if (st != BPDC_OK) return st;
  const bool posterior = p->kp.second_pass_posterior != 0;
  for (int i = 0; i < ncodes; ++i) {
    CodePlan& cp = p->per_code[i];
    bpdc_code c = codes[i];
    if (kernel == BPDC_KERNEL_PLAIN) {
      cp.kernel = BPDC_KERNEL_PLAIN;
      continue;
    }
    const int rule = p->kp.rule;
    std::string why_lane, why_group;
    const bool soft = p->kp.soft_period > 0;
    const bool lane_ok = bpdc::lane_eligible(c->g, posterior, lane_max_lanes(), rule, soft, &why_lane);
    const bool group_ok = group_fits(p.get(), c->dev, &why_group);
    if (kernel == BPDC_KERNEL_LANE) {
      if ((st = choose_lane(p.get(), i, true, &cp, nullptr)) != BPDC_OK) return st;
      cp.kernel = BPDC_KERNEL_LANE;
      cp.chose = "lane (requested)";
      continue;
    }
    if (kernel == BPDC_KERNEL_GROUP) {
      if (!group_ok) return fail(BPDC_ERR_UNSUPPORTED, "group kernel cannot run code %d: %s", i, why_group.c_str());
      if ((st = choose_group_tile(p.get(), i, true, &cp.tile, nullptr, &cp.tried)) != BPDC_OK) return st;
      cp.kernel = BPDC_KERNEL_GROUP;
      cp.chose = "group (requested)";
      continue;
    }
    // AUTO: when both fused families can run the code, each is autotuned on the
    // same kind of synthetic shots and the faster per shot is kept; otherwise
    // the one that can run it (product-sum codes too large for both: plain)
    if (lane_ok && group_ok) {
      double lane_ms = -1.0, group_ms = -1.0;
      if ((st = choose_lane(p.get(), i, true, &cp, &lane_ms)) != BPDC_OK) return st;
      if ((st = choose_group_tile(p.get(), i, true, &cp.tile, nullptr, &cp.tried, &group_ms)) != BPDC_OK) return st;
      if (group_ms > 0 && (lane_ms < 0 || group_ms < lane_ms)) {
        if (cp.lane.mod) (void)hipModuleUnload(cp.lane.mod);
        cp.lane = LaneKernel();
        cp.kernel = BPDC_KERNEL_GROUP;
        cp.chose = "group (faster than lane)";
      } else {
        cp.kernel = BPDC_KERNEL_LANE;
        cp.chose = "lane (faster than group)";
      }
    } else if (lane_ok) {
      if ((st = choose_lane(p.get(), i, true, &cp, nullptr)) != BPDC_OK) return st;
      cp.kernel = BPDC_KERNEL_LANE;
      cp.chose = "lane (group cannot run the code: " + why_group + ")";
    } else if (group_ok) {
      if ((st = choose_group_tile(p.get(), i, true, &cp.tile, nullptr, &cp.tried)) != BPDC_OK) return st;
      cp.kernel = BPDC_KERNEL_GROUP;
      cp.chose = "group (lane cannot run the code: " + why_lane + ")";
    } else if (soft || rule == BPDC_RULE_PRODUCT_SUM) {
      cp.kernel = BPDC_KERNEL_PLAIN;  // too large for one workgroup's LDS, or product-sum rows above 8
      cp.chose = "plain (no fused family can run the code)";
    } else {
      return fail(BPDC_ERR_UNSUPPORTED, "no fused kernel for code %d (lane: %s; group: %s)", i, why_lane.c_str(),
                  why_group.c_str());
    }
  }
  // multi-code launch: the group kernel over all codes, LDS sized for the largest
  p->multi_ok = true;
  {
    int info_bytes = 4;
    size_t lds = 0;
    int maxw = 0;
    for (int i = 0; i < ncodes; ++i) {
      std::string why;
      if (!group_fits(p.get(), codes[i]->dev, &why)) {
        p->multi_ok = false;
        p->multi_why = "code " + std::to_string(i) + ": " + why;
      }
      info_bytes = std::max(info_bytes, code_info_bytes(codes[i]->dev));
      maxw = std::max(maxw, std::max(codes[i]->dev.n, codes[i]->dev.m));
    }
    for (int i = 0; i < ncodes; ++i)
      lds = std::max(lds, bpdc::group_lds_bytes_nm(codes[i]->dev.n, codes[i]->dev.m, group_prior_array(p.get()),
                                                   info_bytes, codes[i]->dev.E));
    if (lds > (size_t)p->max_lds) {
      p->multi_ok = false;
      p->multi_why = "largest per-shot state exceeds the LDS of one workgroup";
    }
    if (p->kp.rule != BPDC_RULE_MIN_SUM) {
      p->multi_ok = false;
      p->multi_why = "the multi-code launch runs scaled min-sum only";
    }
    if (p->multi_ok) {
      bpdc::GroupTile t;
      t.info_bytes = info_bytes;
      t.lds_bytes = lds;
      int th = 64;
      while (th < 512 && th < maxw / 2) th *= 2;
      // autotuned tile of the largest code, when one was chosen
      int big = 0;
      for (int i = 1; i < ncodes; ++i)
        if (codes[i]->dev.n > codes[big]->dev.n) big = i;
      if (p->per_code[big].kernel == BPDC_KERNEL_GROUP) th = p->per_code[big].tile.threads;
      t.threads = th;
      const int nb = bpdc::group_occupancy(th, lds, info_bytes, p->max_lds);
      t.grid = std::max(1, nb) * p->num_cu;
      p->multi_tile = t;
      if (ncodes > 1) {  // a mixed batch: time the thread counts on synthetic shots of every code
        std::vector<int> cands;
        for (int c2 : {256, 512, 1024})
          if (c2 / 2 < maxw) cands.push_back(c2);
        if (cands.empty()) cands.push_back(th);
        if ((st = choose_multi_tile(p.get(), t, cands)) != BPDC_OK) return st;
      }
    }
  }
  *out = p.release();
  return BPDC_OK;
}

bpdc_status bpdc_plan_set_dc_stats(bpdc_plan p, uint64_t* d_stats, int64_t words) {
  if (!p) return fail(BPDC_ERR_INVALID_ARG, "null plan");
  if (d_stats && words < 103) return fail(BPDC_ERR_INVALID_ARG, "DC diagnostics buffer too small");
  p->dcstats = d_stats;
  p->dcstats_words = d_stats ? words : 0;
  return BPDC_OK;
}

bpdc_status bpdc_plan_destroy(bpdc_plan p) {
  if (!p) return BPDC_OK;
  for (auto& cp : p->per_code)
    if (cp.lane.mod) (void)hipModuleUnload(cp.lane.mod);
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->d_code_table) (void)hipFree(p->d_code_table);
  if (p->d_code_by_rank) (void)hipFree(p->d_code_by_rank);
  delete p;
  return BPDC_OK;
}

bpdc_status bpdc_plan_info(bpdc_plan p, int32_t code, int32_t* kernel, int32_t* shots_per_wg,
                           int32_t* threads_per_wg) {
  if (!p || code < 0 || code >= (int)p->per_code.size()) return fail(BPDC_ERR_INVALID_ARG, "bad plan/code");
  const CodePlan& cp = p->per_code[code];
  if (kernel) *kernel = cp.kernel;
  // the lane family runs one wave per workgroup holding 64 / lanes shots; the
  // group family one shot per workgroup; the plain family one shot per thread
  // of its 256-thread phase kernels
  if (shots_per_wg)
    *shots_per_wg = cp.kernel == BPDC_KERNEL_LANE ? 64 / cp.lane.lanes : (cp.kernel == BPDC_KERNEL_GROUP ? 1 : 256);
  if (threads_per_wg)
    *threads_per_wg = cp.kernel == BPDC_KERNEL_LANE ? 64 : (cp.kernel == BPDC_KERNEL_GROUP ? cp.tile.threads : 256);
  return BPDC_OK;
}


bpdc_status bpdc_plan_describe(bpdc_plan p, int32_t code, char* buf, size_t cap, size_t* needed) {
  if (!p || code < -1 || code >= (int)p->per_code.size()) return fail(BPDC_ERR_INVALID_ARG, "bad plan/code");
  std::string o;
  if (code == -1) {
    if (!p->multi_ok) {
      o = "{\"multi_code\": false, \"why\": " + json_str(p->multi_why) + "}";
    } else {
      const bpdc::GroupTile& t = p->multi_tile;
      o = "{\"multi_code\": true, \"threads_per_wg\": " + std::to_string(t.threads) +
          ", \"shots_per_wg\": 1, \"lds_bytes_per_wg\": " + std::to_string(t.lds_bytes) +
          ", \"workgroups\": " + std::to_string(t.grid) + ", \"tried\": " + json_tried(p->multi_tried) + "}";
    }
  } else {
    const CodePlan& cp = p->per_code[code];
    const char* fam = cp.kernel == BPDC_KERNEL_LANE ? "lane" : (cp.kernel == BPDC_KERNEL_GROUP ? "group" : "plain");
    o = "{\"kernel\": \"" + std::string(fam) + "\", \"chose\": " + json_str(cp.chose);
    if (cp.kernel == BPDC_KERNEL_LANE)
      o += ", \"lanes_per_shot\": " + std::to_string(cp.lane.lanes) + ", \"shots_per_wg\": " +
           std::to_string(64 / cp.lane.lanes) + ", \"threads_per_wg\": 64, \"claim_chunk\": " +
           std::to_string(cp.lane.chunk) + ", \"workgroups\": " + std::to_string(cp.lane.grid);
    else if (cp.kernel == BPDC_KERNEL_GROUP)
      o += ", \"threads_per_wg\": " + std::to_string(cp.tile.threads) + ", \"shots_per_wg\": 1, \"lds_bytes\": " +
           std::to_string(cp.tile.lds_bytes) + ", \"workgroups\": " + std::to_string(cp.tile.grid);
    o += ", \"tried\": " + json_tried(cp.tried) + "}";
  }
  if (needed) *needed = o.size() + 1;
  if (buf && cap > 0) {
    const size_t k = std::min(cap - 1, o.size());
    memcpy(buf, o.data(), k);
    buf[k] = 0;
  }
  return BPDC_OK;
}

bpdc_status bpdc_workspace_size(bpdc_plan p, int32_t code, int64_t B, size_t* bytes) {
  if (!p || !bytes || B < 0) return fail(BPDC_ERR_INVALID_ARG, "bad arguments");
  if (code == -1) {
    *bytes = multi_ws_bytes(p, B);
    return BPDC_OK;
  }
  if (code < 0 || code >= (int)p->per_code.size()) return fail(BPDC_ERR_INVALID_ARG, "bad code index");
  const CodePlan& cp = p->per_code[code];
  switch (cp.kernel) {
    case BPDC_KERNEL_PLAIN: *bytes = bpdc::plain_workspace_bytes(p->codes[code]->dev, B); break;
    case BPDC_KERNEL_LANE: *bytes = lane_ws_bytes(cp.lane, B); break;
    default: *bytes = kLaneWs; break;
  }
  return BPDC_OK;
}

bpdc_status bpdc_decode(bpdc_plan p, int32_t code, const uint64_t* d_syn, int64_t B, int64_t shot_offset,
                        uint64_t* d_corr, uint8_t* d_flags, float* d_post, uint64_t* d_cut, int16_t* d_iters,
                        void* d_ws, size_t ws_bytes, void* stream) {
  if (!p) return fail(BPDC_ERR_INVALID_ARG, "null plan");
  if (code < 0 || code >= (int)p->per_code.size()) return fail(BPDC_ERR_INVALID_ARG, "bad code index");
  if (B < 0 || shot_offset < 0) return fail(BPDC_ERR_INVALID_ARG, "negative batch or offset");
  if (B == 0) return BPDC_OK;
  if (!d_syn || !d_corr || !d_flags) return fail(BPDC_ERR_INVALID_ARG, "null syndrome/correction/flags");
  size_t need = 0;
  bpdc_status st = bpdc_workspace_size(p, code, B, &need);
  if (st != BPDC_OK) return st;
  if (!d_ws || ws_bytes < need) return fail(BPDC_ERR_WORKSPACE, "workspace of %zu bytes needed", need);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != p->device) return fail(BPDC_ERR_INVALID_ARG, "plan was created on device %d, current is %d", p->device, dev);
  const CodePlan& cp = p->per_code[code];
  bpdc_code c = p->codes[code];
  if (p->dcstats) {
    if (p->dcstats_words < 103 + c->g.n)
      return fail(BPDC_ERR_INVALID_ARG, "DC diagnostics buffer needs %d words", 103 + c->g.n);
  }
  bpdc::DecodeIO io{d_syn, B, shot_offset, d_corr, d_flags, d_post, d_cut, d_iters, p->dcstats};
  hipStream_t s = (hipStream_t)stream;
  switch (cp.kernel) {
    case BPDC_KERNEL_PLAIN:
      HIP_TRY(bpdc::plain_decode(c->dev, p->kp, io, d_ws, s));
      return BPDC_OK;
    case BPDC_KERNEL_LANE:
      return lane_launch(p, cp, c, io, d_ws, s);
    case BPDC_KERNEL_GROUP: {
      const char* tab = (const char*)p->d_code_table + (size_t)code * sizeof(bpdc::GCodeHost);
      HIP_TRY(bpdc::group_launch(tab, nullptr, nullptr, nullptr, p->kp, d_syn, nullptr, d_corr, nullptr, d_flags, d_post,
                                 d_cut, d_iters, B, shot_offset, cp.tile.threads, cp.tile.grid, cp.tile.lds_bytes,
                                 cp.tile.info_bytes, (unsigned long long*)d_ws, s,
                                 (unsigned long long*)p->dcstats, c->g.n));
      return BPDC_OK;
    }
    default:
      return fail(BPDC_ERR_UNSUPPORTED, "kernel family not available");
  }
}

bpdc_status bpdc_decode_noalloc(bpdc_plan p, int32_t code, const uint64_t* d_syn, int64_t B,
                                int64_t shot_offset, uint64_t* d_corr, uint8_t* d_flags, float* d_post,
                                uint64_t* d_cut, int16_t* d_iters, void* stream) {
  if (!p) return fail(BPDC_ERR_INVALID_ARG, "null plan");
  if (code < 0 || code >= (int)p->per_code.size()) return fail(BPDC_ERR_INVALID_ARG, "bad code index");
  if (B < 0 || shot_offset < 0) return fail(BPDC_ERR_INVALID_ARG, "negative batch or offset");
  size_t need = 0;
  bpdc_status st = bpdc_workspace_size(p, code, B, &need);
  if (st != BPDC_OK) return st;
  if (need > (size_t)BPDC_NOALLOC_SCRATCH_BYTES)
    return fail(BPDC_ERR_WORKSPACE,
                "a batch of %lld shots needs %zu bytes of workspace, above the %zu-byte static scratch of "
                "bpdc_decode_noalloc: decode it in smaller batches or pass a workspace to bpdc_decode",
                (long long)B, need, (size_t)BPDC_NOALLOC_SCRATCH_BYTES);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != p->device) return fail(BPDC_ERR_INVALID_ARG, "plan was created on device %d, current is %d", p->device, dev);
  void* ws = nullptr;
  HIP_TRY(bpdc::noalloc_scratch(dev, &ws));
  return bpdc_decode(p, code, d_syn, B, shot_offset, d_corr, d_flags, d_post, d_cut, d_iters, ws,
                     (size_t)BPDC_NOALLOC_SCRATCH_BYTES, stream);
}

bpdc_status bpdc_decode_multi(bpdc_plan p, const int32_t* d_code_of_shot, const uint64_t* d_syn,
                              const int64_t* d_syn_off, uint64_t* d_corr, const int64_t* d_corr_off,
                              uint8_t* d_flags, int16_t* d_iters, int64_t B, int64_t shot_offset, void* d_ws,
                              size_t ws_bytes, void* stream) {
  if (!p) return fail(BPDC_ERR_INVALID_ARG, "null plan");
  if (B < 0 || shot_offset < 0) return fail(BPDC_ERR_INVALID_ARG, "negative batch or offset");
  if (B == 0) return BPDC_OK;
  if (B > 0x7fffffff) return fail(BPDC_ERR_INVALID_ARG, "multi-code batch above 2^31 shots");
  if (!d_code_of_shot || !d_syn || !d_syn_off || !d_corr || !d_corr_off || !d_flags)
    return fail(BPDC_ERR_INVALID_ARG, "null pointer");
  if (!p->multi_ok) return fail(BPDC_ERR_UNSUPPORTED, "multi-code launch unavailable: %s", p->multi_why.c_str());
  if (p->dcstats) {
    int nmax = 0;
    for (bpdc_code c : p->codes) nmax = std::max(nmax, c->g.n);
    if (p->dcstats_words < 103 + nmax)
      return fail(BPDC_ERR_INVALID_ARG, "DC diagnostics buffer needs %d words (largest code)", 103 + nmax);
  }
  if (!d_ws || ws_bytes < multi_ws_bytes(p, B))
    return fail(BPDC_ERR_WORKSPACE, "workspace of %zu bytes needed", multi_ws_bytes(p, B));
  return multi_enqueue(p, d_code_of_shot, d_syn, d_syn_off, d_corr, d_corr_off, d_flags, d_iters, B, shot_offset,
                       d_ws, (hipStream_t)stream, nullptr, (unsigned long long*)p->dcstats);
}

bpdc_status bpdc_graph_capture_multi(bpdc_plan p, const int32_t* d_code_of_shot, const uint64_t* d_syn,
                                     const int64_t* d_syn_off, uint64_t* d_corr, const int64_t* d_corr_off,
                                     uint8_t* d_flags, int16_t* d_iters, int64_t B, int64_t shot_offset,
                                     void* d_ws, size_t ws_bytes, void* stream) {
  if (!p) return fail(BPDC_ERR_INVALID_ARG, "null plan");
  if (B <= 0 || shot_offset < 0 || B > 0x7fffffff) return fail(BPDC_ERR_INVALID_ARG, "bad batch size");
  if (!d_code_of_shot || !d_syn || !d_syn_off || !d_corr || !d_corr_off || !d_flags)
    return fail(BPDC_ERR_INVALID_ARG, "null pointer");
  if (!p->multi_ok) return fail(BPDC_ERR_UNSUPPORTED, "multi-code launch unavailable: %s", p->multi_why.c_str());
  if (p->dcstats) return fail(BPDC_ERR_UNSUPPORTED, "a captured graph keeps no DC diagnostics");
  if (!d_ws || ws_bytes < multi_ws_bytes(p, B))
    return fail(BPDC_ERR_WORKSPACE, "workspace of %zu bytes needed", multi_ws_bytes(p, B));
  hipStream_t s = (hipStream_t)stream;
  hipStream_t cs = s;
  bool own = false;
  if (!cs) {  // the null stream cannot be captured: capture on a private stream
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    own = true;
  }
  if (p->graph_exec) {
    (void)hipGraphExecDestroy(p->graph_exec);
    p->graph_exec = nullptr;
  }
  if (p->graph) {
    (void)hipGraphDestroy(p->graph);
    p->graph = nullptr;
  }
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  bpdc_status st = BPDC_OK;
  if (e == hipSuccess) {
    st = multi_enqueue(p, d_code_of_shot, d_syn, d_syn_off, d_corr, d_corr_off, d_flags, d_iters, B, shot_offset,
                       d_ws, cs);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (st == BPDC_OK && e2 != hipSuccess) st = fail(BPDC_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e2));
    if (st == BPDC_OK) {
      p->graph = g;
      const hipError_t e3 = hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0);
      if (e3 != hipSuccess) st = fail(BPDC_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e3));
    } else if (g) {
      (void)hipGraphDestroy(g);
    }
  } else {
    st = fail(BPDC_ERR_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  if (own) (void)hipStreamDestroy(cs);
  return st;
}

bpdc_status bpdc_eval_phi(const float* d_x, int64_t n, float* d_out, void* stream) {
  if (n < 0 || (n > 0 && (!d_x || !d_out))) return fail(BPDC_ERR_INVALID_ARG, "bad arguments");
  HIP_TRY(bpdc::eval_phi(d_x, n, d_out, (hipStream_t)stream));
  return BPDC_OK;
}

bpdc_status bpdc_graph_launch(bpdc_plan p, void* stream) {
  if (!p) return fail(BPDC_ERR_INVALID_ARG, "null plan");
  if (!p->graph_exec) return fail(BPDC_ERR_INVALID_ARG, "no graph captured on this plan");
  HIP_TRY(hipGraphLaunch(p->graph_exec, (hipStream_t)stream));
  return BPDC_OK;
}

// ---- weighted min-sum -------------------------------------------------------------------------

static bpdc_status wms_check(bpdc_plan p, int32_t code, int64_t B, int32_t K) {
  if (!p) return fail(BPDC_ERR_INVALID_ARG, "null plan");
  if (code < 0 || code >= (int)p->codes.size()) return fail(BPDC_ERR_INVALID_ARG, "bad code index");
  if (B < 0) return fail(BPDC_ERR_INVALID_ARG, "negative batch");
  if (K < 1) return fail(BPDC_ERR_INVALID_ARG, "ckpt_every must be >= 1");
  if (p->kp.second_pass_posterior)
    return fail(BPDC_ERR_UNSUPPORTED, "weighted min-sum supports the channel second-pass prior only");
  if (p->kp.rule != BPDC_RULE_MIN_SUM) return fail(BPDC_ERR_UNSUPPORTED, "weighted decoding is min-sum only");
  if (p->kp.soft_period > 0) return fail(BPDC_ERR_UNSUPPORTED, "weighted decoding has no soft DC");
  const bpdc::DevCode& d = p->codes[code]->dev;
  if (d.max_row_deg > bpdc::kWmsMaxRowDeg)
    return fail(BPDC_ERR_UNSUPPORTED, "weighted min-sum: rows of at most %d edges (code has %d)", bpdc::kWmsMaxRowDeg,
                d.max_row_deg);
  if (bpdc::wms_backward_lds(d, K) > (size_t)p->max_lds || bpdc::wms_forward_lds(d) > (size_t)p->max_lds)
    return fail(BPDC_ERR_UNSUPPORTED, "code too large for the weighted min-sum kernels (LDS)");
  return BPDC_OK;
}

static size_t wms_ckpt_bytes(bpdc_plan p, int32_t code, int64_t B, int32_t K) {
  return bpdc::wms_ckpt_bytes(p->codes[code]->dev, p->kp, B, K);
}

bpdc_status bpdc_wms_ckpt_size(bpdc_plan p, int32_t code, int64_t B, int32_t K, size_t* bytes) {
  bpdc_status st = wms_check(p, code, B, K);
  if (st != BPDC_OK) return st;
  if (!bytes) return fail(BPDC_ERR_INVALID_ARG, "null bytes");
  *bytes = wms_ckpt_bytes(p, code, B, K);
  return BPDC_OK;
}

bpdc_status bpdc_wms_forward(bpdc_plan p, int32_t code, const float* d_w, const uint64_t* d_syn, int64_t B,
                             int64_t shot_offset, int32_t K, float* d_post, uint64_t* d_cut, uint8_t* d_flags,
                             void* d_ckpt, size_t ckpt_bytes, void* stream) {
  bpdc_status st = wms_check(p, code, B, K);
  if (st != BPDC_OK) return st;
  if (B == 0) return BPDC_OK;
  if (shot_offset < 0) return fail(BPDC_ERR_INVALID_ARG, "negative shot offset");
  if (!d_w || !d_syn || !d_post || !d_cut || !d_flags) return fail(BPDC_ERR_INVALID_ARG, "null pointer");
  if (!d_ckpt || ckpt_bytes < wms_ckpt_bytes(p, code, B, K))
    return fail(BPDC_ERR_WORKSPACE, "checkpoint buffer of %zu bytes needed", wms_ckpt_bytes(p, code, B, K));
  HIP_TRY(bpdc::wms_forward(p->codes[code]->dev, p->kp, d_w, d_syn, B, shot_offset, K, d_post, d_cut, d_flags,
                            d_ckpt, p->num_cu, p->max_lds, (hipStream_t)stream));
  return BPDC_OK;
}

bpdc_status bpdc_wms_backward(bpdc_plan p, int32_t code, const float* d_w, const uint64_t* d_syn, int64_t B,
                              int32_t K, const float* d_grad_post, const uint64_t* d_cut, const uint8_t* d_flags,
                              const void* d_ckpt, size_t ckpt_bytes, float* d_grad_w, void* stream) {
  bpdc_status st = wms_check(p, code, B, K);
  if (st != BPDC_OK) return st;
  if (B == 0) return BPDC_OK;
  if (!d_w || !d_syn || !d_grad_post || !d_cut || !d_flags || !d_grad_w)
    return fail(BPDC_ERR_INVALID_ARG, "null pointer");
  if (!d_ckpt || ckpt_bytes < wms_ckpt_bytes(p, code, B, K))
    return fail(BPDC_ERR_WORKSPACE, "checkpoint buffer of %zu bytes needed", wms_ckpt_bytes(p, code, B, K));
  HIP_TRY(bpdc::wms_backward(p->codes[code]->dev, p->kp, d_w, d_syn, B, K, d_grad_post, d_cut, d_flags,
                             d_ckpt, d_grad_w, p->num_cu, p->max_lds, (hipStream_t)stream));
  return BPDC_OK;
}

}  // extern "C"

