// Host harness for the FP64 log and exp of the sampling path (the library's own
// header, built with the host compiler and -ffp-contract=off, so it evaluates
// exactly the operations the device does): the largest error in units of the
// last place against the x87 extended-precision logl / expl, over the whole
// positive range and densely near 1 for log, over [-745, 0] and near 0 for exp,
// and the special values.  Prints one line per range, "max_ulp <range> <value>",
// then "ok" or the first failing special value (exit status 1).
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <cstdio>

#include "r1_math.hpp"

namespace {

uint64_t rs = 0x2545F4914F6CDD1Dull;
double uniform() {  // [0, 1)
  rs ^= rs << 13;
  rs ^= rs >> 7;
  rs ^= rs << 17;
  return double(rs >> 11) * 0x1p-53;
}

double ulps(double got, long double ref) {
  if (std::isinf(double(ref))) return got == double(ref) ? 0.0 : INFINITY;
  int e;
  std::frexp(double(ref), &e);
  const double ulp = std::ldexp(1.0, std::max(e - 53, -1074));
  return double(std::fabs((long double)got - ref)) / ulp;
}

template <typename F, typename G, typename R>
double max_ulp(const char* name, int n, G gen, F f, R ref) {
  double worst = 0.0, at = 0.0;
  for (int i = 0; i < n; ++i) {
    const double x = gen();
    const double u = ulps(f(x), ref(x));
    if (u > worst) { worst = u; at = x; }
  }
  std::printf("max_ulp %s %.3f at %.17g\n", name, worst, at);
  return worst;
}

}  // namespace

int main() {
  auto lg = [](double x) { return r1x::log_f64(x); };
  auto lgr = [](double x) { return logl((long double)x); };
  auto ex = [](double v) { return r1x::exp_f64(v); };
  auto exr = [](double v) { return expl((long double)v); };
  const int n = 2000000;
  double w = 0.0;
  w = std::fmax(w, max_ulp("log_all", n, [] { return std::ldexp(1.0 + uniform(), int(uniform() * 2097) - 1074); }, lg, lgr));
  w = std::fmax(w, max_ulp("log_near1", n, [] { return 0.5 + 1.5 * uniform(); }, lg, lgr));
  w = std::fmax(w, max_ulp("log_1pm", n, [] { return 1.0 + (uniform() - 0.5) * 1e-6; }, lg, lgr));
  const double wl = w;
  w = 0.0;
  w = std::fmax(w, max_ulp("exp_neg", n, [] { return -745.0 * uniform(); }, ex, exr));
  w = std::fmax(w, max_ulp("exp_unit", n, [] { return -uniform(); }, ex, exr));
  w = std::fmax(w, max_ulp("exp_small", n, [] { return (uniform() - 0.5) * 1e-6; }, ex, exr));
  w = std::fmax(w, max_ulp("exp_pos", n, [] { return 700.0 * uniform(); }, ex, exr));
  const double we = w;
  struct Case { double got, want; const char* what; };
  const double inf = HUGE_VAL;
  const Case cases[] = {
      {r1x::log_f64(0.0), -inf, "log 0"},
      {r1x::log_f64(inf), inf, "log inf"},
      {r1x::log_f64(1.0), 0.0, "log 1"},
      {r1x::exp_f64(0.0), 1.0, "exp 0"},
      {r1x::exp_f64(-inf), 0.0, "exp -inf"},
      {r1x::exp_f64(-800.0), 0.0, "exp -800"},
  };
  for (const Case& c : cases)
    if (!(c.got == c.want)) {
      std::printf("special %s: %.17g\n", c.what, c.got);
      return 1;
    }
  if (!std::isnan(r1x::log_f64(-1.0)) || !std::isnan(r1x::log_f64(NAN)) || !std::isnan(r1x::exp_f64(NAN))) {
    std::printf("special NaN\n");
    return 1;
  }
  std::printf("ok log %.3f exp %.3f\n", wl, we);
  return 0;
}
