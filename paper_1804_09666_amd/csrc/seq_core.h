// seq_core.h -- the sequential NPDM / NTDM sweeps of one system, walked by
// one lane (Veneva & Ayriyan, arXiv:1804.09666, Sec. 1: the LU of the band
// matrix without pivoting, then forward and back substitution).
//
// Every expression is evaluated in the bracketed order of the recurrences,
// with IEEE division and no contraction into FMAs, so pivots, factors, x and
// the breakdown row are the sequential method's to the last bit.  Used by the
// one-lane kernels and by the split-row kernels to redo, sequentially, the
// systems whose partitioned elimination meets a bad or tiny pivot.
#pragma once

#include <climits>

#include "bs_internal.h"
#include "lane_stream.h"

namespace bs {
namespace seq {

constexpr int kPF = 8;  // rows in flight per lane (6 loads per row, < 64 outstanding)

// Transient info value inside one call: the system waits for the sequential
// redo (never left in info when the call's launches have completed).
constexpr int32_t kRedo = INT_MIN;

// Redo slots of a separate redo launch: each slot holds the np planes of one
// system of up to nmax rows; at most 256 slots and about 256 MB of planes.
inline int64_t redo_slots(int64_t np, int64_t nmax, int64_t count) {
  int64_t r = (int64_t(1) << 25) / (np * (nmax > 0 ? nmax : 1));
  if (r > 256) r = 256;
  if (r > count) r = count;
  return r < 1 ? 1 : r;
}

struct Row {
  double e, c, d, a, b, y;
};

__device__ inline bool bad_pivot(double m) { return !(m != 0.0) || !isfinite(m); }

// Per-row state of the forward sweep for the backward one: row i of column
// col at al[i * pitch + col] (and be, z likewise; be unused for NTDM).  z may
// be the x array itself (zpitch = its leading dimension) when x is FP64 and
// no other writer touches the system's x.
struct Planes {
  double* al;
  double* be;
  int64_t pitch;
  double* z;
  int64_t zpitch;
  int64_t col;
};

// NPDM (KIND 5):
//   gamma_i = c_i - alpha_{i-2} e_i,   mu_i = (d_i - beta_{i-2} e_i) - alpha_{i-1} gamma_i,
//   alpha_i = (a_i - beta_{i-1} gamma_i) / mu_i,   beta_i = b_i / mu_i,
//   z_i = ((y_i - z_{i-2} e_i) - z_{i-1} gamma_i) / mu_i,
//   x_i = (z_i - alpha_i x_{i+1}) - beta_i x_{i+2};
// NTDM (KIND 3): mu_i = d_i - alpha_{i-1} c_i, alpha_i = a_i / mu_i,
//   z_i = (y_i - z_{i-1} c_i) / mu_i, x_i = z_i - alpha_i x_{i+1}.
// Terms whose index falls outside the matrix are omitted, so the corner
// slots are never used.  fetch(i) returns row i (called up to kPF rows
// ahead; rows are in [0, n)); put(i, v) stores x_i when keep(i) holds.  The
// sweeps run on past a bad pivot (x is then unspecified); returns the first
// bad row, or -1.
template <int KIND, typename Fetch, typename Put, typename Keep>
__device__ int64_t solve(int64_t n, Fetch&& fetch, const Planes& P, Put&& put, Keep&& keep) {
#pragma clang fp contract(off)
  int64_t bad = -1;
  {
    double am1 = 0, am2 = 0, bm1 = 0, bm2 = 0, zm1 = 0, zm2 = 0;
    Row ring[kPF];
    auto get = [&](int q, int64_t i) { ring[q] = fetch(i); };
    auto use = [&](int q, int64_t i) {
      const Row& w = ring[q];
      double gamma = 0, mu, ali = 0, bei = 0, zi;
      if (KIND == 5) {
        if (i == 0) {
          mu = w.d;
        } else if (i == 1) {
          gamma = w.c;
          mu = w.d - am1 * gamma;
        } else {
          gamma = w.c - am2 * w.e;
          mu = (w.d - bm2 * w.e) - am1 * gamma;
        }
        if (i <= n - 2) ali = (i == 0) ? w.a / mu : (w.a - bm1 * gamma) / mu;
        if (i <= n - 3) bei = w.b / mu;
        if (i == 0)
          zi = w.y / mu;
        else if (i == 1)
          zi = (w.y - zm1 * gamma) / mu;
        else
          zi = ((w.y - zm2 * w.e) - zm1 * gamma) / mu;
      } else {
        if (i == 0) {
          mu = w.d;
        } else {
          gamma = w.c;
          mu = w.d - am1 * gamma;
        }
        if (i <= n - 2) ali = w.a / mu;
        zi = (i == 0) ? w.y / mu : (w.y - zm1 * gamma) / mu;
      }
      if (bad < 0 && bad_pivot(mu)) bad = i;
      P.al[i * P.pitch + P.col] = ali;
      if (KIND == 5) P.be[i * P.pitch + P.col] = bei;
      P.z[i * P.zpitch + P.col] = zi;
      am2 = am1;
      am1 = ali;
      bm2 = bm1;
      bm1 = bei;
      zm2 = zm1;
      zm1 = zi;
    };
    stream_rows<kPF, false>(n, get, use);
  }
  {
    double rz[kPF], ral[kPF], rbe[kPF];
    double xp1 = 0, xp2 = 0;  // x_{i+1}, x_{i+2}
    auto get = [&](int q, int64_t i) {
      rz[q] = P.z[i * P.zpitch + P.col];
      ral[q] = P.al[i * P.pitch + P.col];
      rbe[q] = (KIND == 5) ? P.be[i * P.pitch + P.col] : 0.0;
    };
    auto use = [&](int q, int64_t i) {
      double xi;
      if (i == n - 1)
        xi = rz[q];
      else if (KIND == 3 || i == n - 2)
        xi = rz[q] - ral[q] * xp1;
      else
        xi = (rz[q] - ral[q] * xp1) - rbe[q] * xp2;
      if (keep(i)) put(i, xi);
      xp2 = xp1;
      xp1 = xi;
    };
    stream_rows<kPF, true>(n, get, use);
  }
  return bad;
}

}  // namespace seq
}  // namespace bs
