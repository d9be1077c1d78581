// Host-only driver of the plan code (plan.cpp) for an AddressSanitizer / UBSan build: plans
// of every form and dtype over the workload bands, queries, delay tables, time binning,
// and the argument errors. Exits non-zero on a failed check; the sanitizers abort on misuse.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../include/dedisp.h"

static int failures = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

static std::vector<double> band(double f_top, double bw, int nchan) {
  std::vector<double> f(nchan);
  for (int c = 0; c < nchan; ++c) f[c] = f_top - c * (bw / nchan);
  return f;
}

static std::vector<double> dms(double step, int n) {
  std::vector<double> d(n);
  for (int i = 0; i < n; ++i) d[i] = i * step;
  return d;
}

int main() {
  struct Case {
    double f_top, bw, tsamp, step;
    int nchan, ndm;
  } cases[] = {{428, 20, 51.2e-6, 0.1, 64, 128},    {428, 20, 51.2e-6, 0.1, 1024, 2048},
               {180, 60, 81.92e-6, 0.05, 4096, 512}, {428, 20, 51.2e-6, 0.2, 256, 700},
               {428, 20, 51.2e-6, 0.1, 1, 1},        {428, 20, 51.2e-6, 0.3, 37, 33}};
  for (const Case& k : cases) {
    const std::vector<double> f = band(k.f_top, k.bw, k.nchan), d = dms(k.step, k.ndm);
    for (int dtype : {DD_F32, DD_F16, DD_U8})
      for (int form : {DD_FORM_AUTO, DD_FORM_LDS, DD_FORM_REGWIN}) {
        dd_tuning t{};
        t.kernel_form = form;
        dd_plan* p = nullptr;
        const int rc = dd_plan_create(&p, f.data(), k.nchan, k.tsamp, d.data(), k.ndm, dtype, &t);
        if (rc != DD_OK) {
          CHECK(rc == DD_ERR_UNSUPPORTED && p == nullptr);
          continue;
        }
        dd_plan_info info{};
        const int q = dd_plan_query(p, 1 << 20, &info);
        CHECK(q == DD_OK || q == DD_ERR_TOO_SHORT);
        CHECK(info.nchan == k.nchan && info.ndm == k.ndm);
        std::vector<int32_t> tab((size_t)k.nchan * k.ndm);
        CHECK(dd_plan_delays(p, tab.data()) == DD_OK);
        CHECK(tab[0] == 0 && info.maxdelay >= tab.back());
        dd_plan_destroy(p);
      }
    std::vector<int32_t> lg(k.ndm);
    double diag = 0;
    CHECK(dd_time_binning(f.data(), k.nchan, k.tsamp, d.data(), k.ndm, 4, &diag, lg.data()) == DD_OK);
    for (int i = 1; i < k.ndm; ++i) CHECK(lg[i] >= lg[i - 1]);
  }
  // argument errors leave no plan behind
  const std::vector<double> f = band(428, 20, 8), d = dms(0.1, 8);
  dd_plan* p = reinterpret_cast<dd_plan*>(0x1);
  CHECK(dd_plan_create(&p, f.data(), 0, 51.2e-6, d.data(), 8, DD_F32, nullptr) == DD_ERR_INVALID_ARG && !p);
  std::vector<double> bad(d);
  bad[3] = -1.0;
  CHECK(dd_plan_create(&p, f.data(), 8, 51.2e-6, bad.data(), 8, DD_F32, nullptr) == DD_ERR_INVALID_ARG);
  bad[3] = std::nan("");
  CHECK(dd_plan_create(&p, f.data(), 8, 51.2e-6, bad.data(), 8, DD_F32, nullptr) == DD_ERR_INVALID_ARG);
  CHECK(dd_plan_create(&p, f.data(), 8, -1.0, d.data(), 8, DD_F32, nullptr) == DD_ERR_INVALID_ARG);
  dd_tuning t{};
  t.dms_per_wave = 3;
  CHECK(dd_plan_create(&p, f.data(), 8, 51.2e-6, d.data(), 8, DD_F32, &t) == DD_ERR_UNSUPPORTED);
  CHECK(std::string(dd_last_error()).size() > 0);
  dd_plan_destroy(nullptr);
  if (failures) std::fprintf(stderr, "%d checks failed\n", failures);
  else std::printf("asan plan driver: ok\n");
  return failures ? 1 : 0;
}
