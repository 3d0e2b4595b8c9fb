// Resonance peaks and the H-infinity norm estimate of a model on the
// imaginary axis, from frequency-response evaluations with derivatives.
//
// sigma(w) = sigma_max(G(j w)).  Where the largest singular value is simple,
// with G(jw) v1 = sigma u1,
//     d sigma / d w = Re(u1^H (dG/dw) v1),  dG/dw = j dG/ds
// (first-order perturbation of a simple singular value; e.g. Stewart & Sun,
// Matrix Perturbation Theory, 1990, ch. IV).  The caller's grid is evaluated
// once (G and dG/ds on the float64 path); each local maximum of sigma on it
// is bracketed by its grid neighbours, and the zero of d sigma / d w inside
// the bracket is found by a safeguarded secant iteration (a secant step when
// it stays inside the bracket, else bisection), all peaks advancing together
// with one request per iteration.  The estimate of ||G||_inf is the largest
// of the refined peaks, the grid values and sigma_max(D) (w -> infinity).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "lti_freqresp.h"

namespace {

using cd = std::complex<double>;

// Largest singular value of the p x m matrix G (row-major) and its singular
// vectors, by one-sided Jacobi (Hestenes) on the columns of G (or of G^H when
// m > p): rotate column pairs until every pair is orthogonal; then the
// column norms are the singular values and the accumulated rotations the
// right singular vectors.
struct Top {
  double s;
  std::vector<cd> u, v;  // G v = s u, |u| = |v| = 1
};

Top sigma_max(const cd* G, int p, int m) {
  const bool tr = m > p;
  const int r = tr ? m : p, c = tr ? p : m;  // work on W (r x c), r >= c
  std::vector<cd> W((size_t)r * c), V((size_t)c * c, cd(0.0));
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < c; ++j) W[(size_t)i * c + j] = tr ? std::conj(G[(size_t)j * m + i]) : G[(size_t)i * m + j];
  for (int j = 0; j < c; ++j) V[(size_t)j * c + j] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int a = 0; a < c - 1; ++a)
      for (int b = a + 1; b < c; ++b) {
        double aa = 0.0, bb = 0.0;
        cd ab = 0.0;
        for (int i = 0; i < r; ++i) {
          const cd x = W[(size_t)i * c + a], y = W[(size_t)i * c + b];
          aa += std::norm(x);
          bb += std::norm(y);
          ab += std::conj(x) * y;
        }
        const double g = std::abs(ab);
        if (g == 0.0 || g <= 1e-17 * std::sqrt(aa * bb)) continue;
        off = std::max(off, g / std::sqrt(aa * bb));
        // the 2x2 Hermitian [[aa, ab], [conj(ab), bb]] is diagonalised by
        // [[c, -s conj(e)], [s e, c]] with e = ab / |ab|
        const cd e = ab / g;
        const double zeta = (bb - aa) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::abs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
        for (int i = 0; i < r; ++i) {
          const cd x = W[(size_t)i * c + a], y = W[(size_t)i * c + b];
          W[(size_t)i * c + a] = cs * x - sn * std::conj(e) * y;
          W[(size_t)i * c + b] = sn * e * x + cs * y;
        }
        for (int i = 0; i < c; ++i) {
          const cd x = V[(size_t)i * c + a], y = V[(size_t)i * c + b];
          V[(size_t)i * c + a] = cs * x - sn * std::conj(e) * y;
          V[(size_t)i * c + b] = sn * e * x + cs * y;
        }
      }
    if (off <= 1e-15) break;
  }
  int best = 0;
  double bn = -1.0;
  for (int j = 0; j < c; ++j) {
    double nn = 0.0;
    for (int i = 0; i < r; ++i) nn += std::norm(W[(size_t)i * c + j]);
    if (nn > bn) {
      bn = nn;
      best = j;
    }
  }
  Top t;
  t.s = std::sqrt(std::max(bn, 0.0));
  std::vector<cd> left(r), right(c);
  for (int i = 0; i < r; ++i) left[i] = t.s > 0 ? W[(size_t)i * c + best] / t.s : cd(i == 0 ? 1.0 : 0.0);
  for (int i = 0; i < c; ++i) right[i] = V[(size_t)i * c + best];
  // W = M V with M = G (or G^H): M right = s left
  if (tr) {  // G^H right = s left  =>  G left = s right
    t.u = right;
    t.v = left;
  } else {
    t.u = left;
    t.v = right;
  }
  return t;
}

struct Eval {
  std::vector<double> sig, dsig;
};

std::atomic<uint64_t> g_key{0};

// G and dG/ds at the points w (one request through the context), then
// sigma_max and d sigma / d w at each.
int evaluate(lti_ctx* c, const lti_request& base, const std::vector<double>& w, uint64_t key, Eval& ev) {
  const int p = base.ny, m = base.nu;
  const size_t K = w.size();
  std::vector<double> G(2 * K * p * m), dG(2 * K * p * m);
  lti_request q = base;
  q.mem = LTI_MEM_HOST;
  q.omega = w.data();
  q.n_omega = (int64_t)K;
  q.points = LTI_POINTS_JW;
  q.precision = LTI_PREC_FP64;
  q.model_key = key;
  q.G_out = G.data();
  q.dG_out = dG.data();
  q.info_out = nullptr;
  uint64_t id = 0;
  int rc = lti_freqresp_submit(c, &q, &id);
  if (rc != LTI_OK) return rc;
  lti_result res{};
  rc = lti_freqresp_poll(c, id, -1, &res);
  if (rc != LTI_OK) return rc;
  ev.sig.resize(K);
  ev.dsig.resize(K);
  const cd* Gc = reinterpret_cast<const cd*>(G.data());
  const cd* dGc = reinterpret_cast<const cd*>(dG.data());
  for (size_t k = 0; k < K; ++k) {
    const Top t = sigma_max(Gc + k * p * m, p, m);
    // Re(u^H (j dG/ds) v)
    cd acc = 0.0;
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < m; ++j) acc += std::conj(t.u[i]) * dGc[k * p * m + (size_t)i * m + j] * t.v[j];
    ev.sig[k] = t.s;
    ev.dsig[k] = std::real(cd(0.0, 1.0) * acc);
  }
  return LTI_OK;
}

}  // namespace

extern "C" int lti_freqresp_peaks(lti_ctx* c, const lti_request* req, int32_t max_peaks, double wtol,
                                  lti_peak* peaks, lti_hinf_result* out) {
  if (!c || !req || !out || max_peaks < 0 || (max_peaks > 0 && !peaks)) return LTI_EINVAL;
  if (req->mem != LTI_MEM_HOST || req->points != LTI_POINTS_JW || req->n_omega < 1 || !req->omega)
    return LTI_EINVAL;
  if (!(wtol > 0.0)) wtol = 1e-12;
  std::memset(out, 0, sizeof(*out));
  // a private key keeps the reduced model resident across the iterations
  const uint64_t key = (uint64_t(1) << 63) | (0x5EA4ull << 40) | ++g_key;
  std::vector<double> w(req->omega, req->omega + req->n_omega);
  std::sort(w.begin(), w.end());
  w.erase(std::unique(w.begin(), w.end()), w.end());
  Eval ev;
  int rc = evaluate(c, *req, w, key, ev);
  if (rc != LTI_OK) return rc;
  int64_t evals = (int64_t)w.size();
  const size_t K = w.size();
  // the H-infinity candidates: every grid value, and sigma_max(D) at w -> inf
  double hinf = 0.0, whinf = 0.0;
  for (size_t k = 0; k < K; ++k)
    if (ev.sig[k] > hinf) {
      hinf = ev.sig[k];
      whinf = w[k];
    }
  if (req->D) {
    std::vector<cd> D((size_t)req->ny * req->nu);
    for (size_t i = 0; i < D.size(); ++i) D[i] = req->D[i];
    const double sd = sigma_max(D.data(), req->ny, req->nu).s;
    if (sd > hinf) {
      hinf = sd;
      whinf = INFINITY;
    }
  }
  // interior local maxima of the grid, largest first
  struct Br {
    double lo, hi, flo, fhi, best_w, best_s;
  };
  std::vector<std::pair<double, size_t>> loc;
  for (size_t k = 1; k + 1 < K; ++k)
    if (ev.sig[k] >= ev.sig[k - 1] && ev.sig[k] >= ev.sig[k + 1] && ev.sig[k] > 0.0) loc.emplace_back(ev.sig[k], k);
  std::sort(loc.begin(), loc.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
  if ((int)loc.size() > max_peaks) loc.resize(max_peaks);
  std::vector<Br> br;
  for (const auto& l : loc) {
    const size_t k = l.second;
    br.push_back(Br{w[k - 1], w[k + 1], ev.dsig[k - 1], ev.dsig[k + 1], w[k], ev.sig[k]});
  }
  // safeguarded secant on d sigma / d w = 0 inside each bracket (f >= 0 at
  // lo, f <= 0 at hi); all brackets advance together
  for (int it = 0; it < 60 && !br.empty(); ++it) {
    std::vector<double> wn;
    std::vector<size_t> who;
    for (size_t i = 0; i < br.size(); ++i) {
      Br& b = br[i];
      if (b.hi - b.lo <= wtol * std::max(std::abs(b.best_w), 1e-300)) continue;
      double x = 0.5 * (b.lo + b.hi);
      if (b.flo > 0.0 && b.fhi < 0.0) {
        const double sec = b.lo - b.flo * (b.hi - b.lo) / (b.fhi - b.flo);
        // keep the step away from the ends, so the bracket shrinks
        const double margin = 0.01 * (b.hi - b.lo);
        if (sec > b.lo + margin && sec < b.hi - margin) x = sec;
      }
      wn.push_back(x);
      who.push_back(i);
    }
    if (wn.empty()) break;
    Eval e2;
    rc = evaluate(c, *req, wn, key, e2);
    if (rc != LTI_OK) return rc;
    evals += (int64_t)wn.size();
    for (size_t q = 0; q < wn.size(); ++q) {
      Br& b = br[who[q]];
      if (e2.sig[q] > b.best_s) {
        b.best_s = e2.sig[q];
        b.best_w = wn[q];
      }
      if (e2.dsig[q] > 0.0) {
        b.lo = wn[q];
        b.flo = e2.dsig[q];
      } else {
        b.hi = wn[q];
        b.fhi = e2.dsig[q];
      }
    }
  }
  std::sort(br.begin(), br.end(), [](const Br& a, const Br& b) { return a.best_s > b.best_s; });
  for (size_t i = 0; i < br.size(); ++i) {
    peaks[i].w = br[i].best_w;
    peaks[i].gain = br[i].best_s;
    if (br[i].best_s > hinf) {
      hinf = br[i].best_s;
      whinf = br[i].best_w;
    }
  }
  out->hinf = hinf;
  out->w_hinf = whinf;
  out->n_peaks = (int32_t)br.size();
  out->evaluations = (int32_t)std::min<int64_t>(evals, INT32_MAX);
  return LTI_OK;
}
