// C ABI of the frequency-domain EMRI mode sum: argument validation,
// context-owned scratch memory and the launch sequence
//   spline coefficients -> mode constants + piece table -> bin-major gather.
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <fstream>
#include <mutex>
#include <sstream>
#include <vector>

#include "fdemri_internal.hpp"

namespace fdemri {
hipError_t launch_spline(int K, const double* t, const double* Fphi, const double* Fr, const double* Phiphi,
                         const double* Phir, const double* A, int Nm, double* tcoef, double* acoef, double* fac,
                         int32_t* status, hipStream_t stream);
size_t spline_factor_doubles(int K);
struct PieceArgs;
hipError_t launch_setup_flat(int K, int Nm, int Nf, const double* t, const double* Fphi, const double* Fr,
                             const double* f, const double* tcoef, const int32_t* l, const int32_t* m,
                             const int32_t* n, double theta, double phi, double scale, uint32_t flags,
                             const double* A, double* acoef, float* acoef32, double* fac, ModeConst* modes,
                             float4* modes32, int2* mode_kr, Piece* pieces, int64_t* evals, int32_t* status,
                             uint32_t* flag_word, const double* Phiphi, const double* Phir, const double* A_in,
                             int hann, bool grouped, bool combine, int2* gkr, int32_t* gsize, GroupMember* gmem,
                             GroupMember32* gmem32, hipStream_t stream);
bool setup_fusable(int K, int Nm, int Nf, uint32_t flags);
hipError_t launch_setup_fused(int K, int Nm, int Nf, const double* t, const double* Fphi, const double* Fr,
                              const double* Phiphi, const double* Phir, const double* f, double* tcoef,
                              const int32_t* l, const int32_t* m, const int32_t* n, double theta, double phi,
                              double scale, uint32_t flags, const double* A, double* acoef, float* acoef32,
                              ModeConst* modes, float4* modes32, int2* mode_kr, Piece* pieces, int64_t* evals,
                              int32_t* slots, uint32_t* flag_word, const double* A_in, int hann,
                              hipStream_t stream);
struct GatherArgs;
hipError_t launch_gather_flat(const Prepared& p, const float* acoef32, void* hp, void* hc, bool mixed, int bpl,
                              hipStream_t stream);
int spline_blocks(int n_series);
hipError_t launch_spline_batch(const WaveItem* items, int B, const int32_t* block_prefix, int total_blocks, int Kmax,
                               hipStream_t stream);
hipError_t launch_amp32(int Nm, int K, const double* t, const double* acoef, float* acoef32, hipStream_t stream);
hipError_t launch_amp32_batch(const WaveItem* items, int B, const int32_t* amp_prefix, int total, hipStream_t stream);
hipError_t launch_pieces_batch(const WaveItem* items, int B, const int32_t* mode_prefix, int total_modes,
                               const int32_t* check_prefix, int total_checks, int hann, uint32_t* flag_word,
                               hipStream_t stream);
hipError_t launch_gather_batch(const WaveItem* items, int B, const int32_t* item_prefix, int total_items,
                               int* counter, int Kmax, bool mixed, int bpl, hipStream_t stream);
int gather_items_per_waveform(int Nf, int bpl);
hipError_t launch_td(int K, int Nm, const double* t, const double* Phiphi, const double* Phir, const double* tcoef,
                     const double* acoef, const ModeConst* modes, double t0, double dt, int Nt, double* hp, double* hc,
                     hipStream_t stream);
hipError_t launch_trajectory(const void* params, int B, int K, double* out, uint32_t* flag_word, hipStream_t stream);
hipError_t launch_band(int Nm, const ModeConst* modes, const Piece* pieces, double* band, hipStream_t stream);
hipError_t launch_select_modes(int K, int Nm, const double* A, double eps, double* P, int32_t* keep, int32_t* idx,
                               int32_t* n_keep, hipStream_t stream);
int loglike_tiles(int Nf, int bpl);
size_t loglike_partial_doubles(int Nf, int bpl);
int loglike_batch_reduce_blocks(int Nf_max);
hipError_t launch_loglike_batch(const WaveItem* items, int B, const int32_t* item_prefix, int total_items,
                                int* counter, int Kmax, bool mixed, int bpl, int hann, int Nf_max,
                                double* block_sums, double* out, hipStream_t stream);
hipError_t launch_loglike(const Prepared& p, const float* acoef32, bool mixed, int bpl, const void* d_p,
                          const void* d_c, const double* wS, int hann, double* partial, double* edge, double* out,
                          hipStream_t stream);
hipError_t launch_vjp_units(const Prepared& p, const float* acoef32, bool mixed, const void* g_hp, const void* g_hc,
                            double* gA_coef, double* PZ, double* Upart, int2* rng, int32_t* nb, int32_t* off,
                            unsigned long long* ctl, int32_t* unit_of, double* mom, void* scan_tmp,
                            size_t scan_bytes, hipStream_t stream);
size_t vjp_scan_bytes(long units);
long vjp_max_chunks(long units);
size_t vjp_mom_bytes(long units);
hipError_t launch_vjp_reduce(const Prepared& p, double* PZ, double* Upart, double* T3, double* gPhi_coef,
                             double* g_scalars, const int32_t* l, const int32_t* m, double theta, double phi,
                             double scale, uint32_t flags, hipStream_t stream);
hipError_t launch_spa_factor(int n, const double* gd, const double* gdd, const int32_t* dir, void* out, bool mixed,
                             hipStream_t stream);
hipError_t launch_spline_adjoint(int K, const double* t, int Nm, const double* gPhi_coef, const double* gA_coef,
                                 double* gPhi_knots, double* gA_knots, const int32_t* status, hipStream_t stream);
}  // namespace fdemri

using namespace fdemri;

// Fixed scratch of fdemri_waveform_noalloc: one copy per device, resident
// from the module's load to the end of the process.  Host code must not use
// the symbol's name as an address (it names a host-side stand-in); it uses
// the device address that hipGetSymbolAddress returns for the current
// device, kept per device below.
static __device__ __align__(256) char scratch[FDEMRI_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of device dev's copy of `scratch`, looked up once per device
// with dev current (the caller has made it current).
hipError_t scratch_address(int dev, void** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

struct fdemri_ctx {
  int device = 0;
  std::string err;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  uint32_t* flag_word = nullptr;  // device
  // per-mode evaluation counts of the last call, per waveform: the device
  // counts of its Nm rows and, when its rows were grouped, the group sizes
  // and members by sorted position (device)
  struct EvalRecord {
    const int64_t* evals;
    int Nm;
    const int32_t* gsize;
    const GroupMember* gmem;
  };
  std::vector<EvalRecord> last_evals;
  // pinned staging of batch records (reused; guarded by an event)
  char* stage = nullptr;
  size_t stage_bytes = 0;
  hipEvent_t stage_ev = nullptr;
  bool stage_pending = false;
  // batch graphs
  uint32_t flags = 0;
  hipStream_t gstream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  struct GraphEntry {
    std::vector<uint64_t> key;
    hipGraphExec_t exec;
    hipGraph_t graph;
    char* records;     // pinned copy of the batch records read by the graph
    hipEvent_t done;   // recorded after each replay: the records may be rewritten once it has passed
    uint64_t last_use; // for least-recently-used eviction
  };
  std::vector<GraphEntry> graphs;
  uint64_t graph_clock = 0;
  std::vector<char> rec_tmp;  // host image of a batch's records, compared with a graph's
  uint64_t ws_generation = 0;
  // workspaces replaced by a larger one, each with an event recorded on the
  // stream of the call that replaced it; freed once that event has passed
  std::vector<std::pair<char*, hipEvent_t>> retired;
  // autotuned bins-per-lane by (precision, batch?, log2 of total bins)
  std::string device_key;
  std::vector<std::array<int, 4>> tuned;  // {prec, batch, cls, bpl}
  bool tuning = false;                     // the autotuner fixes bpl itself
  int bpl = 4;
  // profiling: event pairs per launch, by kernel class (classes in prof_mask)
  bool prof = false;
  uint32_t prof_mask = (1u << FDEMRI_KERNEL_COUNT) - 1u;
  struct Rec {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  // this device's copy of the fixed scratch (fdemri_waveform_noalloc), or
  // NULL with the lookup's error
  char* scratch = nullptr;
  hipError_t scratch_err = hipSuccess;
  // test hook (FDEMRI_TEST_FAIL_ALLOC=n at fdemri_create): the n-th growth of
  // the workspace fails as a failed device allocation would; 0: off
  int fail_alloc = 0;
};

namespace {

fdemri_status fail(fdemri_ctx* c, fdemri_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return st;
}

fdemri_status hip_fail(fdemri_ctx* c, hipError_t e, const char* what) {
  return fail(c, e == hipErrorOutOfMemory ? FDEMRI_ENOMEM : FDEMRI_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Scratch layout of one waveform.
struct Layout {
  size_t tcoef, fac, acoef, acoef32, modes, modes32, mode_kr, pieces, evals, status, slots;
  size_t gkr, gsize, gmem, gmem32;  // voice groups
  size_t gA, PZ, Upart, T3, gPhi, gsc;  // adjoint scratch (0 bytes unless requested)
  size_t vrng, vnb, voff, vctl, vscan, vunit, vmom, vscan_bytes;  // the adjoint's chunk plan
  size_t ll_partial, ll_edge;           // likelihood scratch (0 bytes unless requested)
  size_t total;
};

// ll_tiles, ll_partial: tiles of the likelihood gather and doubles of its
// partial sums (0: no likelihood scratch).
Layout layout_for(int K, int Nm, bool mixed, bool vjp = false, int ll_tiles = 0, size_t ll_partial = 0) {
  Layout L{};
  size_t off = 0;
  const size_t nseg = (size_t)K - 1;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  L.tcoef = take(4 * nseg * 4 * sizeof(double));
  L.fac = take(spline_factor_doubles(K) * sizeof(double));
  L.acoef = take((size_t)Nm * nseg * 8 * sizeof(double));
  L.acoef32 = take(mixed ? (size_t)Nm * nseg * 8 * sizeof(float) : 0);
  L.modes = take((size_t)Nm * sizeof(ModeConst));
  L.modes32 = take(mixed ? (size_t)Nm * sizeof(float4) : 0);
  L.mode_kr = take((size_t)Nm * sizeof(int2));
  L.pieces = take((size_t)Nm * kMaxPieces * sizeof(Piece));
  L.evals = take((size_t)Nm * sizeof(int64_t));
  L.status = take(4 * sizeof(int32_t));
  L.slots = take(kFusedMaxSlots * sizeof(int32_t));
  const size_t ng = modes_grouped(Nm) ? (size_t)Nm : 0;
  L.gkr = take(ng * sizeof(int2));
  L.gsize = take(ng * sizeof(int32_t));
  L.gmem = take(ng * sizeof(GroupMember));
  L.gmem32 = take(mixed ? ng * sizeof(GroupMember32) : 0);
  const size_t units = vjp ? (size_t)Nm * nseg : 0;
  L.gA = take(units * 8 * sizeof(double));
  L.PZ = take(units * 4 * sizeof(double));
  L.Upart = take(units * 4 * sizeof(double));
  L.T3 = take(vjp ? (size_t)Nm * 4 * sizeof(double) : 0);
  L.gPhi = take(vjp ? 2 * nseg * 4 * sizeof(double) : 0);
  L.gsc = take(vjp ? 8 * sizeof(double) : 0);
  // the chunk plan: per unit its pieces' bin ranges, bins and first chunk;
  // per chunk its unit and moments (at most vjp_max_chunks chunks)
  L.vrng = take(units * kMaxPieces * sizeof(int2));
  L.vnb = take(units * sizeof(int32_t));
  L.voff = take(units * sizeof(int32_t));
  L.vctl = take(vjp ? 2 * sizeof(unsigned long long) : 0);
  L.vscan_bytes = vjp ? vjp_scan_bytes((long)units) : 0;
  L.vscan = take(L.vscan_bytes);
  const size_t max_chunks = vjp ? (size_t)vjp_max_chunks((long)units) : 0;
  L.vunit = take(max_chunks * sizeof(int32_t));
  L.vmom = take(vjp ? vjp_mom_bytes((long)units) : 0);
  L.ll_partial = take(ll_partial * sizeof(double));
  L.ll_edge = take((size_t)ll_tiles * 16 * sizeof(double));
  L.total = off;
  return L;
}

// Frees the retired workspaces whose events have passed (all of them, after
// a synchronisation, when wait is set).
void reclaim_retired(fdemri_ctx* c, bool wait) {
  size_t keep = 0;
  for (auto& r : c->retired) {
    if (wait || hipEventQuery(r.second) == hipSuccess) {
      (void)hipEventSynchronize(r.second);
      (void)hipEventDestroy(r.second);
      (void)hipFree(r.first);
    } else {
      c->retired[keep++] = r;
    }
  }
  c->retired.resize(keep);
}

// Grows the workspace to at least `bytes`.  The old workspace may still be
// read by kernels of earlier calls; calls on a context are ordered (one
// stream, or events), so those kernels finish before any work enqueued on
// `stream` from now on starts.  The old workspace is therefore retired with
// an event recorded on `stream` and freed once the event has passed (checked
// here and at destruction), without synchronising the device or other
// streams.
fdemri_status ensure_ws(fdemri_ctx* c, size_t bytes, hipStream_t stream) {
  reclaim_retired(c, false);
  if (bytes <= c->ws_bytes) return FDEMRI_OK;
  if (c->fail_alloc > 0 && --c->fail_alloc == 0)
    return fail(c, FDEMRI_ENOMEM, "hipMalloc(workspace): out of memory (injected by FDEMRI_TEST_FAIL_ALLOC)");
  const size_t want = align_up(bytes + bytes / 4, 1 << 20);
  char* fresh = nullptr;
  hipError_t e = hipMalloc((void**)&fresh, want);
  if (e != hipSuccess) return hip_fail(c, e, "hipMalloc(workspace)");
  if (c->ws) {
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, stream);
    if (e != hipSuccess) {
      if (ev) (void)hipEventDestroy(ev);
      (void)hipFree(fresh);
      return hip_fail(c, e, "workspace retirement event");
    }
    c->retired.emplace_back(c->ws, ev);
  }
  c->ws = fresh;
  c->ws_bytes = want;
  c->ws_generation++;
  return FDEMRI_OK;
}

int size_class(int64_t bins) { return bins <= 1 ? 0 : (int)std::floor(std::log2((double)bins)); }

// Bins per lane for this call: the autotuned choice for (precision, batch,
// size class) if there is one, else the default.
int choose_bpl(const fdemri_ctx* c, int prec, bool batch, int64_t bins) {
  const int cls = size_class(bins);
  for (const auto& t : c->tuned)
    if (t[0] == prec && t[1] == (int)batch && t[2] == cls) return t[3];
  return 1;  // measured best for both precisions on the 3842-mode workload
}

void load_tune_cache(fdemri_ctx* c) {
  const char* path = std::getenv("FDEMRI_TUNE_CACHE");
  if (!path) return;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    std::istringstream ss(line);
    std::string dev;
    int prec, batch, cls, bpl;
    if (!(ss >> dev >> prec >> batch >> cls >> bpl)) continue;  // malformed lines are ignored
    if (dev != c->device_key || (bpl != 1 && bpl != 2 && bpl != 4)) continue;
    c->tuned.push_back({prec, batch, cls, bpl});
  }
}

fdemri_status validate(fdemri_ctx* c, const fdemri_waveform_desc* d) {
  if (!d) return fail(c, FDEMRI_EINVAL, "desc is NULL");
  if (d->K < 4) return fail(c, FDEMRI_EINVAL, "K=%d: a not-a-knot spline needs K >= 4 knots", d->K);
  if (d->K > kMaxKnots) return fail(c, FDEMRI_ENOTSUP, "K=%d exceeds FDEMRI_MAX_KNOTS=%d", d->K, kMaxKnots);
  if (d->Nm < 1) return fail(c, FDEMRI_EINVAL, "Nm=%d: need at least one mode", d->Nm);
  if (d->Nf < 1) return fail(c, FDEMRI_EINVAL, "Nf=%d: need at least one frequency", d->Nf);
  if (!d->t || !d->Fphi || !d->Fr || !d->Phiphi || !d->Phir || !d->l || !d->m || !d->n || !d->A || !d->f)
    return fail(c, FDEMRI_EINVAL, "NULL input pointer in desc");
  if (!(d->theta == d->theta) || !(d->phi == d->phi) || !(d->scale == d->scale))
    return fail(c, FDEMRI_EINVAL, "theta, phi and scale must not be NaN");
  if (d->flags & ~(uint32_t)(FDEMRI_NO_PARTNERS | FDEMRI_COEFFS_GIVEN))
    return fail(c, FDEMRI_EINVAL, "unknown flags 0x%x", d->flags);
  return FDEMRI_OK;
}

hipEvent_t take_event(fdemri_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Bracket one kernel launch with events when profiling is on.
struct ProfScope {
  fdemri_ctx* c;
  int cls;
  hipStream_t s;
  hipEvent_t a = nullptr;
  ProfScope(fdemri_ctx* c_, int cls_, hipStream_t s_, bool enable = true) : c(c_), cls(cls_), s(s_) {
    if (enable && c->prof && ((c->prof_mask >> cls) & 1u)) {
      a = take_event(c);
      if (a) (void)hipEventRecord(a, s);
    }
  }
  ~ProfScope() {
    if (c->prof && a) {
      hipEvent_t b = take_event(c);
      if (b) {
        (void)hipEventRecord(b, s);
        c->recs.push_back({cls, a, b});
      } else {
        c->pool.push_back(a);
      }
    }
  }
};

}  // namespace

extern "C" {

fdemri_status fdemri_create(fdemri_ctx** out, int hip_device, uint32_t flags) {
  if (!out) return FDEMRI_EINVAL;
  *out = nullptr;
  if (flags & ~(uint32_t)FDEMRI_CTX_BATCH_GRAPHS) return FDEMRI_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) return FDEMRI_EDEVICE;
  fdemri_ctx* c = new (std::nothrow) fdemri_ctx();
  if (!c) return FDEMRI_ENOMEM;
  c->device = hip_device;
  c->flags = flags;
  hipError_t e = hipSetDevice(hip_device);
  if (e == hipSuccess) e = hipMalloc((void**)&c->flag_word, sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemset(c->flag_word, 0, sizeof(uint32_t));
  if (e != hipSuccess) {
    if (c->flag_word) (void)hipFree(c->flag_word);
    delete c;
    return e == hipErrorOutOfMemory ? FDEMRI_ENOMEM : FDEMRI_EDEVICE;
  }
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess) {
      std::string name = std::string(prop.name) + "|" + prop.gcnArchName;
      for (auto& ch : name)
        if (ch == ' ') ch = '_';
      c->device_key = name;
    } else {
      c->device_key = "unknown";
    }
  }
  load_tune_cache(c);
  if (const char* v = std::getenv("FDEMRI_TEST_FAIL_ALLOC")) c->fail_alloc = std::max(0, std::atoi(v));
  // the no-allocation entry point's scratch on this device (the device is
  // current), and room for its bookkeeping, so that it needs no allocation
  {
    void* ptr = nullptr;
    c->scratch_err = scratch_address(hip_device, &ptr);
    c->scratch = (char*)ptr;
    c->last_evals.reserve(1);
  }
  *out = c;
  return FDEMRI_OK;
}

void fdemri_destroy(fdemri_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  reclaim_retired(c, true);
  if (c->ws) (void)hipFree(c->ws);
  if (c->flag_word) (void)hipFree(c->flag_word);
  for (auto& r : c->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto ev : c->pool) (void)hipEventDestroy(ev);
  if (c->stage_ev) (void)hipEventDestroy(c->stage_ev);
  if (c->stage) (void)hipHostFree(c->stage);
  for (auto& g : c->graphs) {
    if (g.done) (void)hipEventDestroy(g.done);
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.graph);
    (void)hipHostFree(g.records);
  }
  if (c->ev_in) (void)hipEventDestroy(c->ev_in);
  if (c->ev_out) (void)hipEventDestroy(c->ev_out);
  if (c->gstream) (void)hipStreamDestroy(c->gstream);
  delete c;
}

const char* fdemri_last_error(const fdemri_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

fdemri_status fdemri_sync_flags(fdemri_ctx* c, hipStream_t stream, uint32_t* flags_out) {
  if (!c || !flags_out) return fail(c, FDEMRI_EINVAL, "NULL argument");
  (void)hipSetDevice(c->device);
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
  uint32_t v = 0;
  e = hipMemcpy(&v, c->flag_word, sizeof v, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemset(c->flag_word, 0, sizeof(uint32_t));
  if (e != hipSuccess) return hip_fail(c, e, "flag word read");
  *flags_out = v;
  return FDEMRI_OK;
}

}  // extern "C"

namespace {

// Enqueue the per-waveform preparation (spline coefficients, mode constants,
// piece table, FP32 amplitude table) into the scratch at w described by L
// (the context's workspace unless given).  prof = false leaves the launches
// unbracketed even while profiling is on (no event is created); hann: the
// input checks also require the Hann kernel's DFT grid; fuse: a gather that
// reads the status slots follows, so a small waveform may have its set-up
// fused into one launch.
fdemri_status prepare(fdemri_ctx* c, const fdemri_waveform_desc* d, bool mixed, const Layout& L, Prepared& p,
                      float*& acoef32, hipStream_t stream, char* w = nullptr, bool prof = true, int hann = 0,
                      bool fuse = false, bool adjoint = false) {
  if (!w) w = c->ws;
  double* tcoef = (double*)(w + L.tcoef);
  // with FDEMRI_COEFFS_GIVEN the caller's coefficients (same layout) are read in place
  const bool given = (d->flags & FDEMRI_COEFFS_GIVEN) != 0;
  double* acoef = given ? const_cast<double*>(d->A) : (double*)(w + L.acoef);
  acoef32 = mixed ? (float*)(w + L.acoef32) : nullptr;
  ModeConst* modes = (ModeConst*)(w + L.modes);
  int2* mode_kr = (int2*)(w + L.mode_kr);
  Piece* pieces = (Piece*)(w + L.pieces);
  int64_t* evals = (int64_t*)(w + L.evals);
  int32_t* status = (int32_t*)(w + L.status);
  int32_t* slots = (int32_t*)(w + L.slots);
  hipError_t e;
  const bool fused = fuse && setup_fusable(d->K, d->Nm, d->Nf, d->flags);
  // voice groups for the forward sum (fuse: with the combined amplitude
  // splines, which replace the first rows' coefficients) and the adjoint
  // (without: it reads every row's own), not for the time-domain sum and the
  // band, and only on the context's own coefficients
  const bool grouped = (fuse || adjoint) && !fused && !given && modes_grouped(d->Nm);
  if (fused) {
    // trajectory splines, pieces, amplitude splines and checks in one launch
    ProfScope ps(c, FDEMRI_KERNEL_PIECES, stream, prof);
    e = launch_setup_fused(d->K, d->Nm, d->Nf, d->t, d->Fphi, d->Fr, d->Phiphi, d->Phir, d->f, tcoef, d->l, d->m,
                           d->n, d->theta, d->phi, d->scale, d->flags, given ? nullptr : d->A, acoef, acoef32,
                           modes, mixed ? (float4*)(w + L.modes32) : nullptr, mode_kr, pieces, evals, slots,
                           c->flag_word, d->A, hann, stream);
    if (e == hipSuccess && mixed && given) e = launch_amp32(d->Nm, d->K, d->t, acoef, acoef32, stream);
    if (e != hipSuccess) return hip_fail(c, e, "set-up kernel launch");
  } else {
    {
      // the trajectory splines first: the piece tables need them
      ProfScope ps(c, FDEMRI_KERNEL_SPLINE, stream, prof);
      e = launch_spline(d->K, d->t, d->Fphi, d->Fr, d->Phiphi, d->Phir, d->A, 0, tcoef, acoef,
                        (double*)(w + L.fac), status, stream);
    }
    if (e != hipSuccess) return hip_fail(c, e, "spline kernel launch");
    {
      // piece tables, amplitude splines (and their FP32 form) and the input
      // checks in one launch
      ProfScope ps(c, FDEMRI_KERNEL_PIECES, stream, prof);
      e = launch_setup_flat(d->K, d->Nm, d->Nf, d->t, d->Fphi, d->Fr, d->f, tcoef, d->l, d->m, d->n, d->theta,
                            d->phi, d->scale, d->flags, given ? nullptr : d->A, acoef, acoef32,
                            (double*)(w + L.fac), modes, mixed ? (float4*)(w + L.modes32) : nullptr, mode_kr,
                            pieces, evals, status, c->flag_word, d->Phiphi, d->Phir, d->A, hann, grouped, fuse,
                            (int2*)(w + L.gkr), (int32_t*)(w + L.gsize), (GroupMember*)(w + L.gmem),
                            mixed ? (GroupMember32*)(w + L.gmem32) : nullptr, stream);
      // given coefficients were not splined: their FP32 form separately
      if (e == hipSuccess && mixed && given) e = launch_amp32(d->Nm, d->K, d->t, acoef, acoef32, stream);
    }
    if (e != hipSuccess) return hip_fail(c, e, "piece kernel launch");
  }
  p.K = d->K;
  p.Nm = d->Nm;
  p.Nf = d->Nf;
  p.t = d->t;
  p.Fphi = d->Fphi;
  p.Fr = d->Fr;
  p.Phiphi = d->Phiphi;
  p.Phir = d->Phir;
  p.f = d->f;
  p.tcoef = tcoef;
  p.acoef = acoef;
  p.modes = modes;
  p.mode_kr = mode_kr;
  p.pieces = pieces;
  p.status = status;
  p.modes32 = mixed ? (const float4*)(w + L.modes32) : nullptr;
  p.gkr = grouped ? (const int2*)(w + L.gkr) : nullptr;
  p.gsize = grouped ? (const int32_t*)(w + L.gsize) : nullptr;
  p.gmem = grouped ? (const GroupMember*)(w + L.gmem) : nullptr;
  p.gmem32 = grouped && mixed ? (const GroupMember32*)(w + L.gmem32) : nullptr;
  p.slots = fused ? slots : nullptr;
  p.nslots = fused ? check_blocks(d->K, d->Nm, d->Nf, d->flags) : 0;
  c->last_evals.assign(1, {evals, d->Nm, p.gsize, p.gmem});
  return FDEMRI_OK;
}

}  // namespace

extern "C" {

fdemri_status fdemri_waveform(fdemri_ctx* c, const fdemri_waveform_desc* d, fdemri_prec prec, void* hp, void* hc,
                              hipStream_t stream) {
  if (!c) return FDEMRI_EINVAL;
  c->err.clear();
  fdemri_status st = validate(c, d);
  if (st != FDEMRI_OK) return st;
  if (prec != FDEMRI_FP64 && prec != FDEMRI_MIXED) return fail(c, FDEMRI_EINVAL, "unknown precision %d", (int)prec);
  if (!hp || !hc) return fail(c, FDEMRI_EINVAL, "NULL output pointer");
  const bool mixed = prec == FDEMRI_MIXED;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  const Layout L = layout_for(d->K, d->Nm, mixed);
  st = ensure_ws(c, L.total, stream);
  if (st != FDEMRI_OK) return st;
  Prepared p;
  float* acoef32 = nullptr;
  st = prepare(c, d, mixed, L, p, acoef32, stream, nullptr, true, 0, true);
  if (st != FDEMRI_OK) return st;
  if (!c->tuning) c->bpl = choose_bpl(c, (int)prec, false, d->Nf);
  {
    ProfScope ps(c, FDEMRI_KERNEL_GATHER, stream);
    e = launch_gather_flat(p, acoef32, hp, hc, mixed, c->bpl, stream);
  }
  if (e != hipSuccess) return hip_fail(c, e, "gather kernel launch");
  return FDEMRI_OK;
}

fdemri_status fdemri_waveform_noalloc(fdemri_ctx* c, const fdemri_waveform_desc* d, fdemri_prec prec, void* hp,
                                      void* hc, hipStream_t stream) {
  if (!c) return FDEMRI_EINVAL;
  c->err.clear();
  fdemri_status st = validate(c, d);
  if (st != FDEMRI_OK) return st;
  if (prec != FDEMRI_FP64 && prec != FDEMRI_MIXED) return fail(c, FDEMRI_EINVAL, "unknown precision %d", (int)prec);
  if (!hp || !hc) return fail(c, FDEMRI_EINVAL, "NULL output pointer");
  const bool mixed = prec == FDEMRI_MIXED;
  const Layout L = layout_for(d->K, d->Nm, mixed);
  if (L.total > (size_t)FDEMRI_NOALLOC_SCRATCH_BYTES)
    return fail(c, FDEMRI_ENOTSUP, "K=%d, Nm=%d (%s) need %zu bytes of scratch, more than the fixed %zu", d->K, d->Nm,
                mixed ? "mixed" : "fp64", L.total, (size_t)FDEMRI_NOALLOC_SCRATCH_BYTES);
  if (!c->scratch) return hip_fail(c, c->scratch_err, "hipGetSymbolAddress(scratch)");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  Prepared p;
  float* acoef32 = nullptr;
  st = prepare(c, d, mixed, L, p, acoef32, stream, c->scratch, false, 0, true);
  if (st != FDEMRI_OK) return st;
  const int bpl = c->tuning ? c->bpl : choose_bpl(c, (int)prec, false, d->Nf);
  e = launch_gather_flat(p, acoef32, hp, hc, mixed, bpl, stream);
  if (e != hipSuccess) return hip_fail(c, e, "gather kernel launch");
  return FDEMRI_OK;
}

fdemri_status fdemri_loglike(fdemri_ctx* c, const fdemri_waveform_desc* d, fdemri_prec prec, const void* d_p,
                             const void* d_c, const double* wS, uint32_t ll_flags, double* out, hipStream_t stream) {
  if (!c) return FDEMRI_EINVAL;
  c->err.clear();
  fdemri_status st = validate(c, d);
  if (st != FDEMRI_OK) return st;
  if (prec != FDEMRI_FP64 && prec != FDEMRI_MIXED) return fail(c, FDEMRI_EINVAL, "unknown precision %d", (int)prec);
  if (!d_p || !d_c || !wS || !out) return fail(c, FDEMRI_EINVAL, "NULL data, weight or output pointer");
  if (ll_flags & ~FDEMRI_LL_HANN) return fail(c, FDEMRI_EINVAL, "unknown likelihood flags 0x%x", ll_flags);
  const bool mixed = prec == FDEMRI_MIXED;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  const int bpl = c->tuning ? c->bpl : choose_bpl(c, (int)prec, false, d->Nf);
  const Layout L = layout_for(d->K, d->Nm, mixed, false, loglike_tiles(d->Nf, bpl), loglike_partial_doubles(d->Nf, bpl));
  st = ensure_ws(c, L.total, stream);
  if (st != FDEMRI_OK) return st;
  Prepared p;
  float* acoef32 = nullptr;
  const int hann = (ll_flags & FDEMRI_LL_HANN) ? 1 : 0;
  st = prepare(c, d, mixed, L, p, acoef32, stream, nullptr, true, hann, true);
  if (st != FDEMRI_OK) return st;
  char* w = c->ws;
  {
    ProfScope ps(c, FDEMRI_KERNEL_GATHER, stream);
    e = launch_loglike(p, acoef32, mixed, bpl, d_p, d_c, wS, (ll_flags & FDEMRI_LL_HANN) ? 1 : 0,
                       (double*)(w + L.ll_partial), (double*)(w + L.ll_edge), out, stream);
  }
  if (e != hipSuccess) return hip_fail(c, e, "likelihood kernel launch");
  return FDEMRI_OK;
}

fdemri_status fdemri_td_waveform(fdemri_ctx* c, const fdemri_waveform_desc* d, double t0, double dt, int32_t Nt,
                                 double* hp_t, double* hc_t, hipStream_t stream) {
  if (!c) return FDEMRI_EINVAL;
  c->err.clear();
  fdemri_status st = validate(c, d);
  if (st != FDEMRI_OK) return st;
  if (Nt < 0 || !std::isfinite(t0) || !std::isfinite(dt) || !(dt > 0.0))
    return fail(c, FDEMRI_EINVAL, "invalid time grid (Nt=%d, dt must be finite and > 0)", Nt);
  if (Nt > 0 && (!hp_t || !hc_t)) return fail(c, FDEMRI_EINVAL, "NULL output pointer");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  const Layout L = layout_for(d->K, d->Nm, false);
  st = ensure_ws(c, L.total, stream);
  if (st != FDEMRI_OK) return st;
  Prepared p;
  float* acoef32 = nullptr;
  st = prepare(c, d, false, L, p, acoef32, stream);
  if (st != FDEMRI_OK) return st;
  {
    ProfScope ps(c, FDEMRI_KERNEL_GATHER, stream);
    e = launch_td(d->K, d->Nm, d->t, d->Phiphi, d->Phir, p.tcoef, p.acoef, p.modes, t0, dt, Nt, hp_t, hc_t, stream);
  }
  if (e != hipSuccess) return hip_fail(c, e, "time-domain kernel launch");
  return FDEMRI_OK;
}

fdemri_status fdemri_trajectory(fdemri_ctx* c, int32_t B, const fdemri_traj_params* params, int32_t K, double* out,
                                hipStream_t stream) {
  if (!c) return FDEMRI_EINVAL;
  c->err.clear();
  if (B < 0 || K < 4 || K > kMaxKnots) return fail(c, FDEMRI_EINVAL, "invalid sizes B=%d K=%d", B, K);
  if (B == 0) return FDEMRI_OK;
  if (!params || !out) return fail(c, FDEMRI_EINVAL, "NULL pointer");
  for (int b = 0; b < B; ++b) {
    const fdemri_traj_params& P = params[b];
    const bool ok = std::isfinite(P.M) && P.M > 0 && std::isfinite(P.mu) && P.mu > 0 && std::isfinite(P.T) &&
                    P.T > 0 && P.e0 >= 0 && P.e0 < 1 && std::isfinite(P.p0) && P.p0 > 6.0 + 2.0 * P.e0 + 0.1 &&
                    std::isfinite(P.Phiphi0) && std::isfinite(P.Phir0);
    if (!ok) return fail(c, FDEMRI_EINVAL, "waveform %d: invalid trajectory parameters", b);
  }
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  const size_t bytes = (size_t)B * sizeof(fdemri_traj_params);
  fdemri_status st = ensure_ws(c, bytes, stream);
  if (st != FDEMRI_OK) return st;
  // the parameters go through the workspace; the copy from pageable host
  // memory completes before this call returns
  e = hipMemcpyAsync(c->ws, params, bytes, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(c, e, "parameter upload");
  e = launch_trajectory(c->ws, B, K, out, c->flag_word, stream);
  if (e != hipSuccess) return hip_fail(c, e, "trajectory kernel launch");
  return FDEMRI_OK;
}

fdemri_status fdemri_signal_band(fdemri_ctx* c, const fdemri_waveform_desc* d, double* band, hipStream_t stream) {
  if (!c) return FDEMRI_EINVAL;
  c->err.clear();
  fdemri_status st = validate(c, d);
  if (st != FDEMRI_OK) return st;
  if (!band) return fail(c, FDEMRI_EINVAL, "NULL output pointer");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  const Layout L = layout_for(d->K, d->Nm, false);
  st = ensure_ws(c, L.total, stream);
  if (st != FDEMRI_OK) return st;
  Prepared p;
  float* acoef32 = nullptr;
  st = prepare(c, d, false, L, p, acoef32, stream);
  if (st != FDEMRI_OK) return st;
  e = launch_band(d->Nm, p.modes, p.pieces, band, stream);
  if (e != hipSuccess) return hip_fail(c, e, "band kernel launch");
  return FDEMRI_OK;
}

fdemri_status fdemri_select_modes(fdemri_ctx* c, int32_t K, int32_t Nm, const double* A, double eps, int32_t* idx,
                                  int32_t* n_keep, hipStream_t stream) {
  if (!c) return FDEMRI_EINVAL;
  c->err.clear();
  if (K < 1 || Nm < 0) return fail(c, FDEMRI_EINVAL, "invalid sizes K=%d Nm=%d", K, Nm);
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(c, FDEMRI_EINVAL, "eps must be finite and >= 0");
  if (!n_keep || (Nm > 0 && (!A || !idx))) return fail(c, FDEMRI_EINVAL, "NULL pointer");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  const size_t p_bytes = align_up((size_t)K * sizeof(double), 256);
  fdemri_status st = ensure_ws(c, p_bytes + (size_t)Nm * sizeof(int32_t) + 256, stream);
  if (st != FDEMRI_OK) return st;
  e = launch_select_modes(K, Nm, A, eps, (double*)c->ws, (int32_t*)(c->ws + p_bytes), idx, n_keep, stream);
  if (e != hipSuccess) return hip_fail(c, e, "mode selection launch");
  return FDEMRI_OK;
}

fdemri_status fdemri_vjp(fdemri_ctx* c, const fdemri_waveform_desc* d, fdemri_prec prec, const void* g_hp,
                         const void* g_hc, double* gA, double* gPhi, double* gA_knots, double* gPhi_knots,
                         double* g_scalars, hipStream_t stream) {
  if (!c) return FDEMRI_EINVAL;
  c->err.clear();
  fdemri_status st = validate(c, d);
  if (st != FDEMRI_OK) return st;
  if (prec != FDEMRI_FP64 && prec != FDEMRI_MIXED) return fail(c, FDEMRI_EINVAL, "unknown precision %d", (int)prec);
  if (gA_knots && (d->flags & FDEMRI_COEFFS_GIVEN))
    return fail(c, FDEMRI_EINVAL, "gA_knots requested but the amplitudes are given as coefficients");
  if (!g_hp || !g_hc) return fail(c, FDEMRI_EINVAL, "NULL cotangent pointer");
  const bool mixed = prec == FDEMRI_MIXED;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  const Layout L = layout_for(d->K, d->Nm, mixed, true);
  st = ensure_ws(c, L.total, stream);
  if (st != FDEMRI_OK) return st;
  Prepared p;
  float* acoef32 = nullptr;
  st = prepare(c, d, mixed, L, p, acoef32, stream, nullptr, true, 0, false, true);
  if (st != FDEMRI_OK) return st;
  char* w = c->ws;
  double* gA_coef = gA ? gA : (double*)(w + L.gA);
  double* gPhi_coef = gPhi ? gPhi : (double*)(w + L.gPhi);
  double* gsc = g_scalars ? g_scalars : (double*)(w + L.gsc);
  {
    // the profiling class brackets the adjoint's bin work (plan, scan, chunks, sums)
    ProfScope ps(c, FDEMRI_KERNEL_VJP, stream);
    e = launch_vjp_units(p, acoef32, mixed, g_hp, g_hc, gA_coef, (double*)(w + L.PZ), (double*)(w + L.Upart),
                         (int2*)(w + L.vrng), (int32_t*)(w + L.vnb), (int32_t*)(w + L.voff),
                         (unsigned long long*)(w + L.vctl), (int32_t*)(w + L.vunit), (double*)(w + L.vmom),
                         w + L.vscan, L.vscan_bytes, stream);
  }
  if (e == hipSuccess)
    e = launch_vjp_reduce(p, (double*)(w + L.PZ), (double*)(w + L.Upart), (double*)(w + L.T3), gPhi_coef, gsc, d->l,
                          d->m, d->theta, d->phi, d->scale, d->flags, stream);
  if (e == hipSuccess && (gA_knots || gPhi_knots))
    e = launch_spline_adjoint(d->K, d->t, d->Nm, gPhi_coef, gA_coef, gPhi_knots, gA_knots, p.status, stream);
  if (e != hipSuccess) return hip_fail(c, e, "vjp kernel launch");
  return FDEMRI_OK;
}

fdemri_status fdemri_spa_factor(fdemri_ctx* c, fdemri_prec prec, int32_t n, const double* gd, const double* gdd,
                                const int32_t* dir, void* G, hipStream_t stream) {
  if (!c) return FDEMRI_EINVAL;
  c->err.clear();
  if (prec != FDEMRI_FP64 && prec != FDEMRI_MIXED) return fail(c, FDEMRI_EINVAL, "unknown precision %d", (int)prec);
  if (n < 0) return fail(c, FDEMRI_EINVAL, "n=%d must be >= 0", n);
  if (n > 0 && (!gd || !gdd || !dir || !G)) return fail(c, FDEMRI_EINVAL, "NULL pointer");
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = launch_spa_factor(n, gd, gdd, dir, G, prec == FDEMRI_MIXED, stream);
  if (e != hipSuccess) return hip_fail(c, e, "special-function kernel launch");
  return FDEMRI_OK;
}

// Sums, over the last call's waveforms, the evaluation counts of all rows
// (groups = false) or of the first row of every voice group (groups = true;
// a waveform whose rows were not grouped counts every row).
static fdemri_status sum_last_evals(fdemri_ctx* c, hipStream_t stream, bool groups, int64_t* count_out) {
  if (!c || !count_out) return fail(c, FDEMRI_EINVAL, "NULL argument");
  if (c->last_evals.empty()) return fail(c, FDEMRI_EINVAL, "no waveform evaluated on this context yet");
  (void)hipSetDevice(c->device);
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
  int64_t s = 0;
  for (const auto& r : c->last_evals) {
    std::vector<int64_t> v(r.Nm);
    e = hipMemcpy(v.data(), r.evals, v.size() * sizeof(int64_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "eval count read");
    if (!groups || !r.gsize) {
      for (int64_t x : v) s += x;
      continue;
    }
    std::vector<int32_t> size(r.Nm);
    std::vector<GroupMember> mem(r.Nm);
    e = hipMemcpy(size.data(), r.gsize, size.size() * sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(mem.data(), r.gmem, mem.size() * sizeof(GroupMember), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "group table read");
    for (int j = 0; j < r.Nm; ++j) {
      const int row = mem[j].mode;
      if (size[j] > 0 && row >= 0 && row < r.Nm) s += v[row];
    }
  }
  *count_out = s;
  return FDEMRI_OK;
}

fdemri_status fdemri_last_eval_count(fdemri_ctx* c, hipStream_t stream, int64_t* count_out) {
  return sum_last_evals(c, stream, false, count_out);
}

fdemri_status fdemri_last_group_eval_count(fdemri_ctx* c, hipStream_t stream, int64_t* count_out) {
  return sum_last_evals(c, stream, true, count_out);
}

}  // extern "C"

namespace {

// Host-side plan of one batch: per-waveform scratch layouts in the workspace
// and the offsets of the device records, prefixes and work counter.
// With ll set the batch computes the fused likelihood: per-waveform partial
// and edge scratch in the layouts, and the stage-1 triples (B x nbmax x 3
// doubles) at ll_off.
struct BatchPlan {
  bool mixed = false, ll = false;
  int B = 0, Kmax = 0, Nf_max = 0, nbmax = 0;
  int64_t n_checks = 0;
  bool given_mixed = false;  // a member with given coefficients in a mixed batch
  int64_t n_series = 0, n_modes = 0, n_amp = 0, n_items = 0;
  std::vector<Layout> Ls;
  std::vector<size_t> base;
  size_t items_off = 0, pref_off = 0, pref_bytes = 0, counter_off = 0, ll_off = 0, total = 0, record_bytes = 0;
};

fdemri_status plan_batch(fdemri_ctx* c, int B, const fdemri_waveform_desc* descs, bool mixed, void* const* hp,
                         void* const* hc, BatchPlan& P, bool ll = false) {
  if (B > 65535) return fail(c, FDEMRI_ENOTSUP, "B=%d: at most 65535 waveforms per batch", B);
  P.mixed = mixed;
  P.ll = ll;
  P.B = B;
  P.Ls.resize(B);
  P.base.resize(B);
  size_t off = 0;
  for (int b = 0; b < B; ++b) {
    fdemri_status st = validate(c, &descs[b]);
    if (st != FDEMRI_OK) return fail(c, st, "waveform %d: %s", b, c->err.c_str());
    if (!ll && (!hp[b] || !hc[b])) return fail(c, FDEMRI_EINVAL, "waveform %d: NULL output pointer", b);
    P.Ls[b] = ll ? layout_for(descs[b].K, descs[b].Nm, mixed, false, loglike_tiles(descs[b].Nf, c->bpl),
                              loglike_partial_doubles(descs[b].Nf, c->bpl))
                 : layout_for(descs[b].K, descs[b].Nm, mixed);
    P.Nf_max = std::max(P.Nf_max, (int)descs[b].Nf);
    P.base[b] = off;
    off = align_up(off + P.Ls[b].total, 256);
    P.Kmax = std::max(P.Kmax, (int)descs[b].K);
    P.n_series += spline_blocks(4 + ((descs[b].flags & FDEMRI_COEFFS_GIVEN) ? 0 : descs[b].Nm));
    P.n_modes += descs[b].Nm;
    P.n_amp += (int64_t)descs[b].Nm * (descs[b].K - 1);
    P.n_items += gather_items_per_waveform(descs[b].Nf, c->bpl);
    P.n_checks += check_blocks(descs[b].K, descs[b].Nm, descs[b].Nf, descs[b].flags);
    if (mixed && (descs[b].flags & FDEMRI_COEFFS_GIVEN)) P.given_mixed = true;
  }
  if (P.n_amp > 0x7fffffff || P.n_items > 0x7fffffff || P.n_series > 0x7fffffff ||
      P.n_modes / 4 + P.n_checks > 0x7fffffff)
    return fail(c, FDEMRI_ENOTSUP, "batch too large for 32-bit work indices");
  P.items_off = off;
  P.pref_off = align_up(P.items_off + (size_t)B * sizeof(WaveItem), 256);
  P.pref_bytes = 5 * (size_t)(B + 1) * sizeof(int32_t);
  P.counter_off = align_up(P.pref_off + P.pref_bytes, 256);
  P.ll_off = P.counter_off + 256;
  P.nbmax = ll ? loglike_batch_reduce_blocks(P.Nf_max) : 0;
  P.total = align_up(P.ll_off + (size_t)B * P.nbmax * 3 * sizeof(double), 256);
  P.record_bytes = (P.pref_off - P.items_off) + P.pref_bytes;
  return FDEMRI_OK;
}

// Fill the device records of the batch into host memory `rec` (record_bytes);
// for a likelihood batch, ll_d_p, ll_d_c, ll_wS hold the data and weights.
void fill_records(fdemri_ctx* c, const BatchPlan& P, const fdemri_waveform_desc* descs, void* const* hp,
                  void* const* hc, char* rec, const void* const* ll_d_p = nullptr,
                  const void* const* ll_d_c = nullptr, const double* const* ll_wS = nullptr) {
  const int B = P.B;
  char* w = c->ws;
  WaveItem* hitems = (WaveItem*)rec;
  int32_t* hpref = (int32_t*)(rec + (P.pref_off - P.items_off));
  int32_t *series_prefix = hpref, *mode_prefix = hpref + (B + 1), *amp_prefix = hpref + 2 * (B + 1),
          *item_prefix = hpref + 3 * (B + 1), *check_prefix = hpref + 4 * (B + 1);
  series_prefix[0] = mode_prefix[0] = amp_prefix[0] = item_prefix[0] = check_prefix[0] = 0;
  c->last_evals.clear();
  for (int b = 0; b < B; ++b) {
    const fdemri_waveform_desc& d = descs[b];
    const Layout& L = P.Ls[b];
    char* wb = w + P.base[b];
    WaveItem it;
    it.K = d.K;
    it.Nm = d.Nm;
    it.Nf = d.Nf;
    it.flags = d.flags;
    it.t = d.t;
    it.Fphi = d.Fphi;
    it.Fr = d.Fr;
    it.Phiphi = d.Phiphi;
    it.Phir = d.Phir;
    it.A = d.A;
    it.f = d.f;
    it.l = d.l;
    it.m = d.m;
    it.n = d.n;
    it.theta = d.theta;
    it.phi = d.phi;
    it.scale = d.scale;
    it.tcoef = (double*)(wb + L.tcoef);
    it.acoef = (d.flags & FDEMRI_COEFFS_GIVEN) ? const_cast<double*>(d.A) : (double*)(wb + L.acoef);
    it.acoef32 = P.mixed ? (float*)(wb + L.acoef32) : nullptr;
    it.modes = (ModeConst*)(wb + L.modes);
    it.modes32 = P.mixed ? (float4*)(wb + L.modes32) : nullptr;
    it.mode_kr = (int2*)(wb + L.mode_kr);
    it.pieces = (Piece*)(wb + L.pieces);
    it.evals = (int64_t*)(wb + L.evals);
    it.status = (int32_t*)(wb + L.status);
    const bool grouped = modes_grouped(d.Nm) && !(d.flags & FDEMRI_COEFFS_GIVEN);
    it.gkr = grouped ? (int2*)(wb + L.gkr) : nullptr;
    it.gsize = grouped ? (int32_t*)(wb + L.gsize) : nullptr;
    it.gmem = grouped ? (GroupMember*)(wb + L.gmem) : nullptr;
    it.gmem32 = grouped && P.mixed ? (GroupMember32*)(wb + L.gmem32) : nullptr;
    it.hp = P.ll ? nullptr : hp[b];
    it.hc = P.ll ? nullptr : hc[b];
    it.d_p = P.ll ? ll_d_p[b] : nullptr;
    it.d_c = P.ll ? ll_d_c[b] : nullptr;
    it.wS = P.ll ? ll_wS[b] : nullptr;
    it.ll_partial = P.ll ? (double*)(wb + L.ll_partial) : nullptr;
    it.ll_edge = P.ll ? (double*)(wb + L.ll_edge) : nullptr;
    hitems[b] = it;
    series_prefix[b + 1] = series_prefix[b] + spline_blocks(4 + ((d.flags & FDEMRI_COEFFS_GIVEN) ? 0 : d.Nm));
    mode_prefix[b + 1] = mode_prefix[b] + d.Nm;
    amp_prefix[b + 1] = amp_prefix[b] + d.Nm * (d.K - 1);
    item_prefix[b + 1] = item_prefix[b] + gather_items_per_waveform(d.Nf, c->bpl);
    check_prefix[b + 1] = check_prefix[b] + check_blocks(d.K, d.Nm, d.Nf, d.flags);
    c->last_evals.push_back({it.evals, d.Nm, it.gsize, it.gmem});
  }
}

// Enqueue record upload and the four batched launches on `stream` (for a
// likelihood batch: the fused gather and its two reduction stages into
// ll_out[B][3], with the Hann kernel when hann is set).
hipError_t enqueue_batch(fdemri_ctx* c, const BatchPlan& P, const char* rec, hipStream_t stream,
                         double* ll_out = nullptr, int hann = 0) {
  char* w = c->ws;
  const int B = P.B;
  const WaveItem* ditems = (const WaveItem*)(w + P.items_off);
  int32_t* dpref = (int32_t*)(w + P.pref_off);
  hipError_t e = hipMemcpyAsync(w + P.items_off, rec, P.record_bytes, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return e;
  {
    ProfScope ps(c, FDEMRI_KERNEL_SPLINE, stream);
    e = launch_spline_batch(ditems, B, dpref, (int)P.n_series, P.Kmax, stream);
  }
  if (e != hipSuccess) return e;
  {
    ProfScope ps(c, FDEMRI_KERNEL_PIECES, stream);
    e = launch_pieces_batch(ditems, B, dpref + (B + 1), (int)P.n_modes, dpref + 4 * (B + 1), (int)P.n_checks, hann,
                            c->flag_word, stream);
    if (e == hipSuccess && P.given_mixed)
      e = launch_amp32_batch(ditems, B, dpref + 2 * (B + 1), (int)P.n_amp, stream);
  }
  if (e != hipSuccess) return e;
  ProfScope ps(c, FDEMRI_KERNEL_GATHER, stream);
  if (P.ll)
    return launch_loglike_batch(ditems, B, dpref + 3 * (B + 1), (int)P.n_items, (int*)(w + P.counter_off), P.Kmax,
                                P.mixed, c->bpl, hann, P.Nf_max, (double*)(w + P.ll_off), ll_out, stream);
  return launch_gather_batch(ditems, B, dpref + 3 * (B + 1), (int)P.n_items, (int*)(w + P.counter_off), P.Kmax,
                             P.mixed, c->bpl, stream);
}

// Key of a batch graph: what the captured launches depend on (precision,
// block shape, sizes, flags and every pointer).  The per-waveform host
// scalars (theta, phi, scale) are not part of it: they only enter the
// records, which a replay reads from the entry's pinned buffer.
std::vector<uint64_t> batch_key(const fdemri_ctx* c, int B, const fdemri_waveform_desc* descs, int prec,
                                void* const* hp, void* const* hc) {
  std::vector<uint64_t> k;
  k.reserve(4 + (size_t)B * 14);
  k.push_back((uint64_t)prec);
  k.push_back((uint64_t)B);
  k.push_back((uint64_t)c->bpl);
  for (int b = 0; b < B; ++b) {
    const fdemri_waveform_desc& d = descs[b];
    k.push_back(((uint64_t)(uint32_t)d.K << 32) | (uint32_t)d.Nm);
    k.push_back(((uint64_t)(uint32_t)d.Nf << 32) | d.flags);
    for (const void* ptr : {(const void*)d.t, (const void*)d.Fphi, (const void*)d.Fr, (const void*)d.Phiphi,
                            (const void*)d.Phir, (const void*)d.l, (const void*)d.m, (const void*)d.n,
                            (const void*)d.A, (const void*)d.f, (const void*)hp[b], (const void*)hc[b]})
      k.push_back((uint64_t)(uintptr_t)ptr);
  }
  return k;
}

// Release one graph entry once its last replay has finished.
void release_graph(fdemri_ctx::GraphEntry& g) {
  if (g.done) {
    (void)hipEventSynchronize(g.done);
    (void)hipEventDestroy(g.done);
  }
  (void)hipGraphExecDestroy(g.exec);
  (void)hipGraphDestroy(g.graph);
  (void)hipHostFree(g.records);
}

void drop_graphs(fdemri_ctx* c) {
  for (auto& g : c->graphs) release_graph(g);
  c->graphs.clear();
}

// Graphs kept per context; the least recently used one is released first.
constexpr size_t kMaxBatchGraphs = 8;

}  // namespace

extern "C" {

fdemri_status fdemri_waveform_batch(fdemri_ctx* c, int32_t B, const fdemri_waveform_desc* descs, fdemri_prec prec,
                                    void* const* hp, void* const* hc, hipStream_t stream) {
  if (!c) return FDEMRI_EINVAL;
  c->err.clear();
  if (B < 0 || (B > 0 && (!descs || !hp || !hc))) return fail(c, FDEMRI_EINVAL, "invalid batch arguments");
  if (B == 0) return FDEMRI_OK;
  if (prec != FDEMRI_FP64 && prec != FDEMRI_MIXED) return fail(c, FDEMRI_EINVAL, "unknown precision %d", (int)prec);
  if (!c->tuning) {
    int64_t bins = 0;
    for (int b = 0; b < B; ++b) bins += descs[b].Nf;
    c->bpl = choose_bpl(c, (int)prec, true, bins);
  }
  BatchPlan P;
  fdemri_status st = plan_batch(c, B, descs, prec == FDEMRI_MIXED, hp, hc, P);
  if (st != FDEMRI_OK) return st;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  const uint64_t gen0 = c->ws_generation;
  st = ensure_ws(c, P.total, stream);
  if (st != FDEMRI_OK) return st;
  if (c->ws_generation != gen0) drop_graphs(c);  // recorded graphs point into the old workspace

  if (!(c->flags & FDEMRI_CTX_BATCH_GRAPHS)) {
    // eager: records through the shared pinned staging buffer
    if (c->stage_pending) {
      e = hipEventSynchronize(c->stage_ev);
      if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize");
      c->stage_pending = false;
    }
    if (P.record_bytes > c->stage_bytes) {
      if (c->stage) (void)hipHostFree(c->stage);
      c->stage = nullptr;
      c->stage_bytes = 0;
      e = hipHostMalloc((void**)&c->stage, P.record_bytes);
      if (e != hipSuccess) return hip_fail(c, e, "hipHostMalloc(staging)");
      c->stage_bytes = P.record_bytes;
    }
    if (!c->stage_ev) {
      e = hipEventCreateWithFlags(&c->stage_ev, hipEventDisableTiming);
      if (e != hipSuccess) return hip_fail(c, e, "hipEventCreate");
    }
    fill_records(c, P, descs, hp, hc, c->stage);
    e = enqueue_batch(c, P, c->stage, stream);
    if (e == hipSuccess) e = hipEventRecord(c->stage_ev, stream);
    if (e != hipSuccess) return hip_fail(c, e, "batch launch");
    c->stage_pending = true;
    return FDEMRI_OK;
  }

  // graph mode: capture once per distinct batch on the context's own stream
  if (!c->gstream) {
    e = hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(c, e, "graph stream set-up");
  }
  const std::vector<uint64_t> key = batch_key(c, B, descs, (int)prec, hp, hc);
  fdemri_ctx::GraphEntry* G = nullptr;
  for (auto& g : c->graphs)
    if (g.key == key) G = &g;
  if (!G) {
    if (c->graphs.size() >= kMaxBatchGraphs) {
      auto lru = std::min_element(c->graphs.begin(), c->graphs.end(),
                                  [](const fdemri_ctx::GraphEntry& a, const fdemri_ctx::GraphEntry& b) {
                                    return a.last_use < b.last_use;
                                  });
      release_graph(*lru);
      c->graphs.erase(lru);
    }
    fdemri_ctx::GraphEntry ne{};
    ne.key = key;
    e = hipEventCreateWithFlags(&ne.done, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventCreate(graph)");
    e = hipHostMalloc((void**)&ne.records, P.record_bytes);
    if (e != hipSuccess) {
      (void)hipEventDestroy(ne.done);
      return hip_fail(c, e, "hipHostMalloc(graph records)");
    }
    fill_records(c, P, descs, hp, hc, ne.records);
    const bool prof = c->prof;
    c->prof = false;
    e = hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal);
    hipError_t e2 = hipSuccess;
    if (e == hipSuccess) e2 = enqueue_batch(c, P, ne.records, c->gstream);
    hipGraph_t graph = nullptr;
    if (e == hipSuccess) e = hipStreamEndCapture(c->gstream, &graph);
    c->prof = prof;
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&ne.exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipHostFree(ne.records);
      (void)hipEventDestroy(ne.done);
      return hip_fail(c, e, "batch graph capture");
    }
    ne.graph = graph;
    c->graphs.push_back(ne);
    G = &c->graphs.back();
  } else {
    // same pointers and shapes: only the host scalars can differ; the
    // records are rewritten (after the entry's last replay has read them)
    // when they do
    c->rec_tmp.resize(P.record_bytes);
    fill_records(c, P, descs, hp, hc, c->rec_tmp.data());
    if (std::memcmp(c->rec_tmp.data(), G->records, P.record_bytes) != 0) {
      e = hipEventSynchronize(G->done);
      if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize(graph)");
      std::memcpy(G->records, c->rec_tmp.data(), P.record_bytes);
    }
  }
  G->last_use = ++c->graph_clock;
  e = hipEventRecord(c->ev_in, stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(c->gstream, c->ev_in, 0);
  if (e == hipSuccess) {
    ProfScope ps(c, FDEMRI_KERNEL_GATHER, c->gstream);
    e = hipGraphLaunch(G->exec, c->gstream);
  }
  if (e == hipSuccess) e = hipEventRecord(G->done, c->gstream);
  if (e == hipSuccess) e = hipEventRecord(c->ev_out, c->gstream);
  if (e == hipSuccess) e = hipStreamWaitEvent(stream, c->ev_out, 0);
  if (e != hipSuccess) return hip_fail(c, e, "batch graph launch");
  return FDEMRI_OK;
}

fdemri_status fdemri_loglike_batch(fdemri_ctx* c, int32_t B, const fdemri_waveform_desc* descs, fdemri_prec prec,
                                   const void* const* d_p, const void* const* d_c, const double* const* wS,
                                   uint32_t ll_flags, double* out, hipStream_t stream) {
  if (!c) return FDEMRI_EINVAL;
  c->err.clear();
  if (B < 0 || (B > 0 && (!descs || !d_p || !d_c || !wS || !out)))
    return fail(c, FDEMRI_EINVAL, "invalid batch arguments");
  if (B == 0) return FDEMRI_OK;
  if (prec != FDEMRI_FP64 && prec != FDEMRI_MIXED) return fail(c, FDEMRI_EINVAL, "unknown precision %d", (int)prec);
  if (ll_flags & ~FDEMRI_LL_HANN) return fail(c, FDEMRI_EINVAL, "unknown likelihood flags 0x%x", ll_flags);
  for (int b = 0; b < B; ++b)
    if (!d_p[b] || !d_c[b] || !wS[b]) return fail(c, FDEMRI_EINVAL, "waveform %d: NULL data or weight pointer", b);
  if (!c->tuning) {
    int64_t bins = 0;
    for (int b = 0; b < B; ++b) bins += descs[b].Nf;
    c->bpl = choose_bpl(c, (int)prec, true, bins);
  }
  BatchPlan P;
  fdemri_status st = plan_batch(c, B, descs, prec == FDEMRI_MIXED, nullptr, nullptr, P, true);
  if (st != FDEMRI_OK) return st;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  const uint64_t gen0 = c->ws_generation;
  st = ensure_ws(c, P.total, stream);
  if (st != FDEMRI_OK) return st;
  if (c->ws_generation != gen0) drop_graphs(c);  // recorded graphs point into the old workspace
  // records through the shared pinned staging buffer (eager; not captured)
  if (c->stage_pending) {
    e = hipEventSynchronize(c->stage_ev);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize");
    c->stage_pending = false;
  }
  if (P.record_bytes > c->stage_bytes) {
    if (c->stage) (void)hipHostFree(c->stage);
    c->stage = nullptr;
    c->stage_bytes = 0;
    e = hipHostMalloc((void**)&c->stage, P.record_bytes);
    if (e != hipSuccess) return hip_fail(c, e, "hipHostMalloc(staging)");
    c->stage_bytes = P.record_bytes;
  }
  if (!c->stage_ev) {
    e = hipEventCreateWithFlags(&c->stage_ev, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventCreate");
  }
  fill_records(c, P, descs, nullptr, nullptr, c->stage, d_p, d_c, wS);
  e = enqueue_batch(c, P, c->stage, stream, out, (ll_flags & FDEMRI_LL_HANN) ? 1 : 0);
  if (e == hipSuccess) e = hipEventRecord(c->stage_ev, stream);
  if (e != hipSuccess) return hip_fail(c, e, "likelihood batch launch");
  c->stage_pending = true;
  return FDEMRI_OK;
}

fdemri_status fdemri_autotune(fdemri_ctx* c, int32_t B, const fdemri_waveform_desc* descs, fdemri_prec prec,
                              void* const* hp, void* const* hc, hipStream_t stream, int32_t* bpl_out) {
  if (!c || B < 1 || !descs || !hp || !hc) return fail(c, FDEMRI_EINVAL, "invalid autotune arguments");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(c, FDEMRI_EDEVICE, "hipEventCreate failed");
  }
  const int cand[3] = {1, 2, 4};
  float best_ms = 1e30f;
  int best = 4;
  c->tuning = true;
  fdemri_status st = FDEMRI_OK;
  for (int ci = 0; ci < 3 && st == FDEMRI_OK; ++ci) {
    c->bpl = cand[ci];
    auto run = [&]() {
      return B == 1 ? fdemri_waveform(c, descs, prec, hp[0], hc[0], stream)
                    : fdemri_waveform_batch(c, B, descs, prec, hp, hc, stream);
    };
    st = run();  // warm-up
    float tot = 0.f;
    for (int r = 0; r < 3 && st == FDEMRI_OK; ++r) {
      (void)hipEventRecord(e0, stream);
      st = run();
      (void)hipEventRecord(e1, stream);
      (void)hipEventSynchronize(e1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      tot += ms;
    }
    if (st == FDEMRI_OK && tot < best_ms) {
      best_ms = tot;
      best = cand[ci];
    }
  }
  c->tuning = false;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != FDEMRI_OK) return st;
  int64_t bins = 0;
  for (int b = 0; b < B; ++b) bins += descs[b].Nf;
  const int batch = B > 1 ? 1 : 0, cls = size_class(bins);
  c->tuned.erase(std::remove_if(c->tuned.begin(), c->tuned.end(),
                                [&](const std::array<int, 4>& t) {
                                  return t[0] == (int)prec && t[1] == batch && t[2] == cls;
                                }),
                 c->tuned.end());
  c->tuned.push_back({(int)prec, batch, cls, best});
  c->bpl = best;
  if (const char* path = std::getenv("FDEMRI_TUNE_CACHE")) {
    std::ofstream out(path, std::ios::app);
    if (out) out << c->device_key << " " << (int)prec << " " << batch << " " << cls << " " << best << "\n";
  }
  if (bpl_out) *bpl_out = best;
  return FDEMRI_OK;
}

fdemri_status fdemri_profile_enable(fdemri_ctx* c, int enable) {
  if (!c) return FDEMRI_EINVAL;
  c->prof = enable != 0;
  return FDEMRI_OK;
}

fdemri_status fdemri_profile_classes(fdemri_ctx* c, uint32_t class_mask) {
  if (!c) return FDEMRI_EINVAL;
  c->err.clear();
  if (class_mask >> FDEMRI_KERNEL_COUNT) return fail(c, FDEMRI_EINVAL, "unknown kernel class in mask 0x%x", class_mask);
  c->prof_mask = class_mask;
  return FDEMRI_OK;
}

fdemri_status fdemri_profile_read(fdemri_ctx* c, hipStream_t stream, double* ms_out, int64_t* launches_out) {
  if (!c || !ms_out || !launches_out) return fail(c, FDEMRI_EINVAL, "NULL argument");
  (void)hipSetDevice(c->device);
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
  for (int k = 0; k < FDEMRI_KERNEL_COUNT; ++k) {
    ms_out[k] = 0.0;
    launches_out[k] = 0;
  }
  for (auto& r : c->recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess && r.cls >= 0 && r.cls < FDEMRI_KERNEL_COUNT) {
      ms_out[r.cls] += ms;
      launches_out[r.cls] += 1;
    }
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->recs.clear();
  return FDEMRI_OK;
}


}  // extern "C"
