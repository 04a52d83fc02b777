// Drives every entry point of the FP64 oracle on small systems so that the
// oracle can run under AddressSanitizer and UndefinedBehaviorSanitizer on
// the CPU (test infrastructure; built and run by tests/test_oracle_native.py).
// The unused corner slots (e_0, e_1, c_0, a_{n-1}, b_{n-2}, b_{n-1}) hold NaN:
// a result that reads them would not be finite.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

extern "C" {
int orc_npdm(int64_t, const double*, const double*, const double*, const double*,
             const double*, const double*, double*, double*);
int orc_ntdm(int64_t, const double*, const double*, const double*, const double*, double*,
             double*);
int orc_mnpdm(int64_t, const double*, const double*, const double*, int64_t, const int64_t*,
              const double*, const double*, const double*, double*);
int orc_ilu0_band(int64_t, const double*, const double*, const double*, const double*,
                  const double*, double*, double*, double*, double*);
int orc_band_lu_solve(int64_t, const double*, const double*, const double*, const double*,
                      const double*, const double*, double*);
int orc_hb_matrix(int64_t, const double*, int, double*);
int orc_hb_lower_apply(int64_t, const double*, const double*, int, const double*, double*);
int orc_hb_upper_apply(int64_t, const double*, const double*, const double*, int,
                       const double*, double*);
int orc_sip(int64_t, const double*, const double*, const double*, const double*, const double*,
            const double*, const double*, const double*, const double*, const double*, double,
            int, int, int, double*, int*, double*);
int orc_dense_solve(int64_t, double*, double*, double*, int);
}

static int failures = 0;
static void check(bool ok, const char* what, int64_t n) {
  if (!ok) {
    std::printf("FAIL %s (n=%lld)\n", what, (long long)n);
    ++failures;
  }
}

int main() {
  std::mt19937_64 gen(1804);
  std::uniform_real_distribution<double> U(-1.0, 1.0), U12(1.0, 2.0);
  const double nan = std::nan("");
  for (int64_t n : {1, 2, 3, 4, 5, 9, 17, 64}) {
    std::vector<double> e(n), c(n), d(n), a(n), b(n), xt(n), y(n, 0.0);
    for (int64_t i = 0; i < n; ++i) {
      e[i] = i >= 2 ? U(gen) : nan;
      c[i] = i >= 1 ? U(gen) : nan;
      a[i] = i <= n - 2 ? U(gen) : nan;
      b[i] = i <= n - 3 ? U(gen) : nan;
      double off = 0.0;
      for (double v : {e[i], c[i], a[i], b[i]})
        if (!std::isnan(v)) off += std::fabs(v);
      d[i] = off + U12(gen);
      xt[i] = U(gen);
    }
    // y = A x_true with the absent terms left out
    for (int64_t i = 0; i < n; ++i) {
      y[i] = d[i] * xt[i];
      if (i >= 2) y[i] += e[i] * xt[i - 2];
      if (i >= 1) y[i] += c[i] * xt[i - 1];
      if (i <= n - 2) y[i] += a[i] * xt[i + 1];
      if (i <= n - 3) y[i] += b[i] * xt[i + 2];
    }
    std::vector<double> x(n), mu(n), x2(n), x3(n);
    check(orc_npdm(n, e.data(), c.data(), d.data(), a.data(), b.data(), y.data(), x.data(),
                   mu.data()) == 0, "npdm info", n);
    double err = 0.0;
    for (int64_t i = 0; i < n; ++i) err = std::fmax(err, std::fabs(x[i] - xt[i]));
    check(err <= 1e-13, "npdm recovers x_true", n);
    // dense Gaussian elimination with partial pivoting on the same matrix
    std::vector<double> A((size_t)(n * n), 0.0), yy(y);
    for (int64_t i = 0; i < n; ++i) {
      A[i * n + i] = d[i];
      if (i >= 2) A[i * n + i - 2] = e[i];
      if (i >= 1) A[i * n + i - 1] = c[i];
      if (i <= n - 2) A[i * n + i + 1] = a[i];
      if (i <= n - 3) A[i * n + i + 2] = b[i];
    }
    std::vector<double> Ad(A);
    check(orc_dense_solve(n, Ad.data(), yy.data(), x2.data(), 1) == 0, "dense info", n);
    err = 0.0;
    for (int64_t i = 0; i < n; ++i) err = std::fmax(err, std::fabs(x[i] - x2[i]));
    check(err <= 1e-13, "npdm = dense", n);
    // tridiagonal part
    std::vector<double> yt(n);
    for (int64_t i = 0; i < n; ++i) {
      yt[i] = d[i] * xt[i];
      if (i >= 1) yt[i] += c[i] * xt[i - 1];
      if (i <= n - 2) yt[i] += a[i] * xt[i + 1];
    }
    check(orc_ntdm(n, c.data(), d.data(), a.data(), yt.data(), x3.data(), mu.data()) == 0,
          "ntdm info", n);
    err = 0.0;
    for (int64_t i = 0; i < n; ++i) err = std::fmax(err, std::fabs(x3[i] - xt[i]));
    check(err <= 1e-13, "ntdm recovers x_true", n);
    // MNPDM with every outer entry listed: bitwise NPDM
    std::vector<int64_t> rows;
    std::vector<double> eat, bat;
    for (int64_t i = 0; i < n; ++i) {
      rows.push_back(i);
      eat.push_back(i >= 2 ? e[i] : 0.0);
      bat.push_back(i <= n - 3 ? b[i] : 0.0);
    }
    std::vector<double> xm(n);
    check(orc_mnpdm(n, c.data(), d.data(), a.data(), n, rows.data(), eat.data(), bat.data(),
                    y.data(), xm.data()) == 0, "mnpdm info", n);
    bool same = true;
    for (int64_t i = 0; i < n; ++i) same = same && xm[i] == x[i];
    check(same, "mnpdm = npdm", n);
    // ILU(0) and its substitution
    std::vector<double> l2(n), l1(n), u0(n), u1(n), xs(n);
    check(orc_ilu0_band(n, e.data(), c.data(), d.data(), a.data(), b.data(), l2.data(),
                        l1.data(), u0.data(), u1.data()) == 0, "ilu0 info", n);
    check(orc_band_lu_solve(n, l2.data(), l1.data(), u0.data(), u1.data(), b.data(), y.data(),
                            xs.data()) == 0, "lu solve info", n);
    err = 0.0;
    for (int64_t i = 0; i < n; ++i) err = std::fmax(err, std::fabs(xs[i] - xt[i]));
    check(err <= 1e-13, "ilu0 + substitution recover x_true", n);
    // HB: vector forms, and the matrix form on the small cases
    std::vector<double> v(n), o1(n), o2(n);
    for (auto& t : v) t = U(gen);
    check(orc_hb_lower_apply(n, l2.data(), l1.data(), 3, v.data(), o1.data()) == 0, "hb lower",
          n);
    check(orc_hb_upper_apply(n, u0.data(), u1.data(), b.data(), 3, v.data(), o2.data()) == 0,
          "hb upper", n);
    for (int64_t i = 0; i < n; ++i)
      check(std::isfinite(o1[i]) && std::isfinite(o2[i]), "hb finite", n);
    if (n <= 17) {
      std::vector<double> X((size_t)(n * n));
      check(orc_hb_matrix(n, A.data(), 2, X.data()) == 0, "hb matrix", n);
    }
    // SIP with HB steps and exact, from zero
    std::vector<double> xsip(n, 0.0);
    int it = -1;
    double rr = -1.0;
    check(orc_sip(n, e.data(), c.data(), d.data(), a.data(), b.data(), y.data(), nullptr,
                  nullptr, nullptr, nullptr, 1e-12, 60, 3, 3, xsip.data(), &it, &rr) == 0,
          "sip hb converges", n);
    std::fill(xsip.begin(), xsip.end(), 0.0);
    check(orc_sip(n, e.data(), c.data(), d.data(), a.data(), b.data(), y.data(), l2.data(),
                  l1.data(), u0.data(), u1.data(), 1e-12, 5, -1, -1, xsip.data(), &it, &rr) == 0,
          "sip exact converges", n);
    // a zero pivot is reported, not divided through
    std::vector<double> dz(d);
    dz[0] = 0.0;
    check(orc_npdm(n, e.data(), c.data(), dz.data(), a.data(), b.data(), y.data(), x.data(),
                   mu.data()) == 1, "zero pivot info", n);
  }
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
