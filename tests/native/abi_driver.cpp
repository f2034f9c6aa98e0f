// Host-side exercise of the C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code of the library's runtime
// (api.hip) and of this driver; the device code is built as usual.
//
//   abi_driver_san nodevice   argument checks that need no GPU: NULL
//                             contexts and arguments, creation on a device
//                             index that does not exist
//   abi_driver_san device     every entry point on device 0 with a small
//                             synthetic waveform, their error returns,
//                             batch graphs, the tuning cache reader on a
//                             malformed file and the allocation-failure hook
//
// Prints one line per step and "abi driver ok" at the end; any failed check
// exits with status 1 (sanitizer reports exit with their own status).
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fdemri.h"

namespace {

int g_fail = 0;

void check(bool ok, const char* what) {
  std::printf("%s %s\n", ok ? "ok  " : "FAIL", what);
  std::fflush(stdout);
  if (!ok) g_fail = 1;
}

#define HIPCHECK(x)                                                            \
  do {                                                                         \
    hipError_t e_ = (x);                                                       \
    if (e_ != hipSuccess) {                                                    \
      std::printf("FAIL %s: %s\n", #x, hipGetErrorString(e_));                 \
      std::exit(1);                                                            \
    }                                                                          \
  } while (0)

template <typename T>
T* dev_copy(const std::vector<T>& h) {
  T* d = nullptr;
  HIPCHECK(hipMalloc((void**)&d, h.size() * sizeof(T)));
  HIPCHECK(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return d;
}

template <typename T>
std::vector<T> host_copy(const T* d, size_t n) {
  std::vector<T> h(n);
  HIPCHECK(hipMemcpy(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost));
  return h;
}

int nodevice() {
  fdemri_waveform_desc d{};
  check(fdemri_waveform(nullptr, &d, FDEMRI_FP64, nullptr, nullptr, nullptr) == FDEMRI_EINVAL,
        "waveform on a NULL context");
  check(fdemri_vjp(nullptr, &d, FDEMRI_FP64, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                   nullptr) == FDEMRI_EINVAL,
        "vjp on a NULL context");
  check(fdemri_profile_enable(nullptr, 1) == FDEMRI_EINVAL, "profile on a NULL context");
  check(std::strlen(fdemri_last_error(nullptr)) > 0, "last error of a NULL context");
  uint32_t fl = 0;
  check(fdemri_sync_flags(nullptr, nullptr, &fl) == FDEMRI_EINVAL, "sync flags on a NULL context");
  int64_t count = 0;
  check(fdemri_last_group_eval_count(nullptr, nullptr, &count) == FDEMRI_EINVAL, "group count on a NULL context");
  fdemri_destroy(nullptr);
  check(fdemri_create(nullptr, 0, 0) != FDEMRI_OK, "create without an output pointer");
  fdemri_ctx* c = nullptr;
  check(fdemri_create(&c, 1 << 20, 0) != FDEMRI_OK && c == nullptr, "create on a device that does not exist");
  return g_fail;
}

// A small synthetic source: K knots over T, slowly chirping fundamental
// frequencies, their phases in closed form, four rows.
struct Source {
  int K = 32, Nm = 4, Nf = 4096;
  double T = 9.3e5;
  std::vector<double> t, Fphi, Fr, Pphi, Pr, A, f;
  std::vector<int32_t> l, m, n;
  Source() {
    const double two_pi = 6.283185307179586;
    for (int i = 0; i < K; ++i) {
      const double ti = T * i / (K - 1);
      t.push_back(ti);
      Fphi.push_back(1e-3 * (1.0 + 0.3 * ti / T));
      Fr.push_back(0.7e-3 * (1.0 + 0.3 * ti / T));
      Pphi.push_back(two_pi * 1e-3 * (ti + 0.15 * ti * ti / T));
      Pr.push_back(0.7 * two_pi * 1e-3 * (ti + 0.15 * ti * ti / T));
    }
    const int rows[4][3] = {{2, 2, 0}, {2, 2, 1}, {3, 3, -1}, {2, 1, 0}};
    for (auto& r : rows) {
      l.push_back(r[0]);
      m.push_back(r[1]);
      n.push_back(r[2]);
    }
    for (int mu = 0; mu < Nm; ++mu)
      for (int i = 0; i < K; ++i) {
        A.push_back((1.0 + 0.2 * mu) * (1.0 + t[i] / T));
        A.push_back(0.1 * (mu + 1));
      }
    for (int k = 0; k < Nf; ++k) f.push_back(k / T);
  }
};

struct DevSource {
  double *t, *Fphi, *Fr, *Pphi, *Pr, *A, *f;
  int32_t *l, *m, *n;
  fdemri_waveform_desc desc{};
  explicit DevSource(const Source& s) {
    t = dev_copy(s.t);
    Fphi = dev_copy(s.Fphi);
    Fr = dev_copy(s.Fr);
    Pphi = dev_copy(s.Pphi);
    Pr = dev_copy(s.Pr);
    A = dev_copy(s.A);
    f = dev_copy(s.f);
    l = dev_copy(s.l);
    m = dev_copy(s.m);
    n = dev_copy(s.n);
    desc.K = s.K;
    desc.t = t;
    desc.Fphi = Fphi;
    desc.Fr = Fr;
    desc.Phiphi = Pphi;
    desc.Phir = Pr;
    desc.Nm = s.Nm;
    desc.l = l;
    desc.m = m;
    desc.n = n;
    desc.A = A;
    desc.theta = 1.0;
    desc.phi = 0.5;
    desc.scale = 1.0;
    desc.Nf = s.Nf;
    desc.f = f;
    desc.flags = 0;
  }
  ~DevSource() {
    for (void* p : {(void*)t, (void*)Fphi, (void*)Fr, (void*)Pphi, (void*)Pr, (void*)A, (void*)f, (void*)l,
                    (void*)m, (void*)n})
      (void)hipFree(p);
  }
};

double rel_l2(const std::vector<double>& a, const std::vector<double>& b) {
  double num = 0.0, den = 0.0;
  for (size_t i = 0; i < a.size(); ++i) {
    num += (a[i] - b[i]) * (a[i] - b[i]);
    den += b[i] * b[i];
  }
  return den > 0.0 ? std::sqrt(num / den) : (num > 0.0 ? 1.0 : 0.0);
}

int device() {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    std::printf("FAIL no device\n");
    return 1;
  }
  // a malformed tuning cache: the reader must skip what it cannot parse
  const char* cache = "abi_driver_tune_cache.txt";
  {
    FILE* fh = std::fopen(cache, "w");
    std::fprintf(fh, "garbage\n|||\nname|arch 0 1 notanumber\n%s\n", std::string(5000, 'x').c_str());
    std::fclose(fh);
  }
  setenv("FDEMRI_TUNE_CACHE", cache, 1);
  fdemri_ctx* c = nullptr;
  check(fdemri_create(&c, 0, FDEMRI_CTX_BATCH_GRAPHS) == FDEMRI_OK && c, "create");
  if (!c) return 1;
  Source s;
  DevSource d(s);
  const int Nf = s.Nf;
  double *hp, *hc, *hp2, *hc2;
  float *mp, *mc;
  HIPCHECK(hipMalloc((void**)&hp, Nf * 16));
  HIPCHECK(hipMalloc((void**)&hc, Nf * 16));
  HIPCHECK(hipMalloc((void**)&hp2, Nf * 16));
  HIPCHECK(hipMalloc((void**)&hc2, Nf * 16));
  HIPCHECK(hipMalloc((void**)&mp, Nf * 8));
  HIPCHECK(hipMalloc((void**)&mc, Nf * 8));
  uint32_t flags = 0;

  check(fdemri_waveform(c, &d.desc, FDEMRI_FP64, hp, hc, nullptr) == FDEMRI_OK, "waveform fp64");
  check(fdemri_sync_flags(c, nullptr, &flags) == FDEMRI_OK && flags == 0, "no flags");
  auto h64 = host_copy(hp, 2 * (size_t)Nf);
  double norm = 0.0;
  bool finite = true;
  for (double v : h64) {
    norm += v * v;
    finite = finite && std::isfinite(v);
  }
  check(finite && norm > 0.0, "fp64 output finite and nonzero");
  int64_t evals = 0;
  check(fdemri_last_eval_count(c, nullptr, &evals) == FDEMRI_OK && evals > 0, "evaluation count");
  int64_t group_evals = 0;
  check(fdemri_last_group_eval_count(c, nullptr, &group_evals) == FDEMRI_OK && group_evals > 0 &&
            group_evals <= evals,
        "group evaluation count");

  check(fdemri_waveform(c, &d.desc, FDEMRI_MIXED, mp, mc, nullptr) == FDEMRI_OK, "waveform mixed");
  {
    auto h32 = host_copy(mp, 2 * (size_t)Nf);
    std::vector<double> h32d(h32.begin(), h32.end());
    check(rel_l2(h32d, h64) <= 1e-5, "mixed against fp64");
  }
  check(fdemri_waveform_noalloc(c, &d.desc, FDEMRI_FP64, hp2, hc2, nullptr) == FDEMRI_OK, "waveform noalloc");
  check(host_copy(hp2, 2 * (size_t)Nf) == h64, "noalloc equals waveform");

  // batch through a captured graph (second call replays it)
  {
    fdemri_waveform_desc ds[3] = {d.desc, d.desc, d.desc};
    void* ph[3] = {hp2, hp2, hp2};
    void* pc[3] = {hc2, hc2, hc2};
    for (int rep = 0; rep < 2; ++rep) {
      HIPCHECK(hipMemset(hp2, 0, Nf * 16));
      check(fdemri_waveform_batch(c, 3, ds, FDEMRI_FP64, ph, pc, nullptr) == FDEMRI_OK, "batch");
      HIPCHECK(hipDeviceSynchronize());
      check(host_copy(hp2, 2 * (size_t)Nf) == h64, "batch equals single call");
    }
  }

  // adjoint with the model as cotangent, likelihood with the model as data
  {
    double *gA, *gPhi, *gAk, *gPk, *gs, *wS, *ll;
    HIPCHECK(hipMalloc((void**)&gA, (size_t)s.Nm * (s.K - 1) * 8 * 8));
    HIPCHECK(hipMalloc((void**)&gPhi, 2 * (size_t)(s.K - 1) * 4 * 8));
    HIPCHECK(hipMalloc((void**)&gAk, (size_t)s.Nm * s.K * 2 * 8));
    HIPCHECK(hipMalloc((void**)&gPk, 2 * (size_t)s.K * 8));
    HIPCHECK(hipMalloc((void**)&gs, 5 * 8));
    check(fdemri_vjp(c, &d.desc, FDEMRI_FP64, hp, hc, gA, gPhi, gAk, gPk, gs, nullptr) == FDEMRI_OK, "vjp");
    auto g = host_copy(gs, 5);
    bool ok = true;
    for (double v : g) ok = ok && std::isfinite(v);
    check(ok, "vjp scalars finite");
    check(fdemri_vjp(c, &d.desc, FDEMRI_FP64, nullptr, hc, gA, gPhi, gAk, gPk, gs, nullptr) == FDEMRI_EINVAL,
          "vjp without a cotangent");
    std::vector<double> w(Nf, 1.0);
    w[0] = 0.0;
    wS = dev_copy(w);
    HIPCHECK(hipMalloc((void**)&ll, 3 * 8));
    check(fdemri_loglike(c, &d.desc, FDEMRI_FP64, hp, hc, wS, FDEMRI_LL_HANN, ll, nullptr) == FDEMRI_OK,
          "loglike");
    auto L = host_copy(ll, 3);
    check(std::isfinite(L[0]) && L[1] > 0.0, "loglike finite");
    check(fdemri_loglike(c, &d.desc, FDEMRI_FP64, hp, hc, nullptr, 0, ll, nullptr) == FDEMRI_EINVAL,
          "loglike without weights");
    for (void* p : {(void*)gA, (void*)gPhi, (void*)gAk, (void*)gPk, (void*)gs, (void*)wS, (void*)ll})
      (void)hipFree(p);
  }

  // trajectories, mode selection, band, time domain, special function
  {
    fdemri_traj_params P[2] = {{1e6, 10.0, 12.0, 0.3, 1e7, 0.0, 0.0}, {1e5, 50.0, 7.0, 0.0, 1e9, 0.1, 0.2}};
    double* out;
    HIPCHECK(hipMalloc((void**)&out, 2 * 7 * 64 * 8));
    check(fdemri_trajectory(c, 2, P, 64, out, nullptr) == FDEMRI_OK, "trajectory");
    fdemri_traj_params bad = P[0];
    bad.p0 = 5.0;
    check(fdemri_trajectory(c, 1, &bad, 64, out, nullptr) == FDEMRI_EINVAL, "trajectory below the plunge");
    check(fdemri_trajectory(c, 1, P, 3, out, nullptr) == FDEMRI_EINVAL, "trajectory with K = 3");
    int32_t *idx, *nk;
    HIPCHECK(hipMalloc((void**)&idx, s.Nm * 4));
    HIPCHECK(hipMalloc((void**)&nk, 4));
    check(fdemri_select_modes(c, s.K, s.Nm, d.A, 1e-3, idx, nk, nullptr) == FDEMRI_OK, "select modes");
    check(fdemri_select_modes(c, s.K, s.Nm, d.A, -1.0, idx, nk, nullptr) == FDEMRI_EINVAL, "select with eps < 0");
    double* band;
    HIPCHECK(hipMalloc((void**)&band, 16));
    check(fdemri_signal_band(c, &d.desc, band, nullptr) == FDEMRI_OK, "signal band");
    double *tp, *tc;
    HIPCHECK(hipMalloc((void**)&tp, 1000 * 8));
    HIPCHECK(hipMalloc((void**)&tc, 1000 * 8));
    check(fdemri_td_waveform(c, &d.desc, 0.0, 900.0, 1000, tp, tc, nullptr) == FDEMRI_OK, "time domain");
    check(fdemri_td_waveform(c, &d.desc, 0.0, -1.0, 1000, tp, tc, nullptr) == FDEMRI_EINVAL, "time domain dt < 0");
    std::vector<double> gd = {1e-9, -2e-10, 0.0}, gdd = {1e-16, 3e-17, 1e-16};
    std::vector<int32_t> dir = {1, -1, 1};
    double *dgd = dev_copy(gd), *dgdd = dev_copy(gdd), *G;
    int32_t* ddir = dev_copy(dir);
    HIPCHECK(hipMalloc((void**)&G, 3 * 16));
    check(fdemri_spa_factor(c, FDEMRI_FP64, 3, dgd, dgdd, ddir, G, nullptr) == FDEMRI_OK, "special function");
    check(fdemri_spa_factor(c, FDEMRI_FP64, -1, dgd, dgdd, ddir, G, nullptr) == FDEMRI_EINVAL,
          "special function n < 0");
    check(fdemri_sync_flags(c, nullptr, &flags) == FDEMRI_OK, "sync after the secondary entry points");
    for (void* p : {(void*)out, (void*)idx, (void*)nk, (void*)band, (void*)tp, (void*)tc, (void*)dgd, (void*)dgdd,
                    (void*)ddir, (void*)G})
      (void)hipFree(p);
  }

  // autotune (appends to the malformed cache) and the profile counters
  {
    void* ph[1] = {hp2};
    void* pc[1] = {hc2};
    int32_t bpl = 0;
    check(fdemri_autotune(c, 1, &d.desc, FDEMRI_FP64, ph, pc, nullptr, &bpl) == FDEMRI_OK && bpl >= 1, "autotune");
    check(fdemri_profile_enable(c, 1) == FDEMRI_OK, "profile on");
    check(fdemri_profile_classes(c, 1u << FDEMRI_KERNEL_GATHER) == FDEMRI_OK, "profile classes");
    check(fdemri_profile_classes(c, 1u << FDEMRI_KERNEL_COUNT) == FDEMRI_EINVAL, "profile class out of range");
    check(fdemri_waveform(c, &d.desc, FDEMRI_FP64, hp, hc, nullptr) == FDEMRI_OK, "profiled waveform");
    double ms[FDEMRI_KERNEL_COUNT];
    int64_t nl[FDEMRI_KERNEL_COUNT];
    check(fdemri_profile_read(c, nullptr, ms, nl) == FDEMRI_OK && nl[FDEMRI_KERNEL_GATHER] == 1, "profile read");
    check(fdemri_profile_enable(c, 0) == FDEMRI_OK, "profile off");
  }
  // a second context reads the cache the first one wrote to
  {
    fdemri_ctx* c2 = nullptr;
    check(fdemri_create(&c2, 0, 0) == FDEMRI_OK && c2, "create after the cache was written");
    fdemri_destroy(c2);
  }

  // argument errors: nothing enqueued, a message on the context
  {
    fdemri_waveform_desc bad = d.desc;
    bad.K = 3;
    check(fdemri_waveform(c, &bad, FDEMRI_FP64, hp, hc, nullptr) == FDEMRI_EINVAL &&
              std::strlen(fdemri_last_error(c)) > 0,
          "K = 3");
    bad = d.desc;
    bad.Nm = 0;
    check(fdemri_waveform(c, &bad, FDEMRI_FP64, hp, hc, nullptr) == FDEMRI_EINVAL, "Nm = 0");
    bad = d.desc;
    bad.f = nullptr;
    check(fdemri_waveform(c, &bad, FDEMRI_FP64, hp, hc, nullptr) == FDEMRI_EINVAL, "NULL grid");
    bad = d.desc;
    bad.theta = NAN;
    check(fdemri_waveform(c, &bad, FDEMRI_FP64, hp, hc, nullptr) == FDEMRI_EINVAL, "NaN angle");
    check(fdemri_waveform(c, &d.desc, (fdemri_prec)7, hp, hc, nullptr) == FDEMRI_EINVAL, "unknown precision");
    check(fdemri_waveform(c, &d.desc, FDEMRI_FP64, nullptr, hc, nullptr) == FDEMRI_EINVAL, "NULL output");
    check(fdemri_waveform(c, nullptr, FDEMRI_FP64, hp, hc, nullptr) == FDEMRI_EINVAL, "NULL descriptor");
    void* ph[1] = {hp};
    void* pc[1] = {hc};
    check(fdemri_waveform_batch(c, -1, &d.desc, FDEMRI_FP64, ph, pc, nullptr) == FDEMRI_EINVAL, "batch B < 0");
    check(fdemri_waveform_batch(c, 0, nullptr, FDEMRI_FP64, nullptr, nullptr, nullptr) == FDEMRI_OK,
          "empty batch");
    check(fdemri_waveform_batch(c, 1, nullptr, FDEMRI_FP64, ph, pc, nullptr) == FDEMRI_EINVAL, "batch NULL descs");
    check(fdemri_waveform(c, &d.desc, FDEMRI_FP64, hp, hc, nullptr) == FDEMRI_OK, "context usable after errors");
  }

  // the allocation-failure hook: the first workspace growth fails
  {
    setenv("FDEMRI_TEST_FAIL_ALLOC", "1", 1);
    fdemri_ctx* c3 = nullptr;
    check(fdemri_create(&c3, 0, 0) == FDEMRI_OK && c3, "create with the failure hook");
    unsetenv("FDEMRI_TEST_FAIL_ALLOC");
    check(fdemri_waveform(c3, &d.desc, FDEMRI_FP64, hp, hc, nullptr) == FDEMRI_ENOMEM, "hooked growth fails");
    check(fdemri_waveform(c3, &d.desc, FDEMRI_FP64, hp, hc, nullptr) == FDEMRI_OK, "next growth succeeds");
    fdemri_destroy(c3);
  }

  HIPCHECK(hipDeviceSynchronize());
  for (void* p : {(void*)hp, (void*)hc, (void*)hp2, (void*)hc2, (void*)mp, (void*)mc}) (void)hipFree(p);
  fdemri_destroy(c);
  std::remove(cache);
  return g_fail;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 2 || (std::strcmp(argv[1], "nodevice") != 0 && std::strcmp(argv[1], "device") != 0)) {
    std::printf("usage: %s nodevice|device\n", argv[0]);
    return 2;
  }
  const int rc = std::strcmp(argv[1], "device") == 0 ? device() : nodevice();
  if (rc == 0) std::printf("abi driver ok\n");
  return rc;
}
