// Host side of the build: w-bin clustering, compute-resource planning and sorting.
//
//  * 1-D k-means (Sect. 3.1): Lloyd iterations on the sorted subset; since bins are
//    intervals between centroid midpoints, each iteration only locates P-1 boundaries
//    by binary search and takes interval means from (long double) prefix sums.
//    Initial centroids at the quantiles floor((p + 1/2) n / P); stop when no boundary
//    moves or after 100 iterations; an empty bin keeps its centroid.
//  * Planner (Sect. 3.4): search P in [1, ceil(P_WSClean)] (eq. 5), estimate K(P) from
//    the planning subset with the kernel-side rule uncapped, evaluate the GPU form of
//    eq. 9 and eq. 10, then the decision tree of Fig. 2.
//  * Subset draw: SplitMix64 (Steele, Lea & Flood 2014) counter-based stream; row k is
//    in the subset iff its k-th output is below f * 2^64.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "wf_internal.h"

namespace wf {

double i0_series(double x) {
  const double q = 0.25 * x * x;
  double term = 1.0, s = 1.0;
  for (int k = 1; k < 300; ++k) {
    term = term * q / ((double)k * (double)k);
    s += term;
    if (term < 1e-18 * s) break;
  }
  return s;
}

// Fourier transform of the Kaiser-Bessel window of support J:
// (J / I0(beta)) sinh(z) / z, z = sqrt(beta^2 - (pi J nu)^2).
double kb_phihat(double nu, int J, double beta) {
  const double a = M_PI * J * nu;
  const double z = std::sqrt(beta * beta - a * a);
  return (J / i0_series(beta)) * std::sinh(z) / z;
}

int nk_rule(double wproj, const KernelParams& kp, bool capped) {
  if (wproj == 0.0) return 1;
  const double lp = ((double)kp.o * kp.Lx) / 2.0;
  const double mp = ((double)kp.o * kp.Ly) / 2.0;
  const double nn = std::sqrt(1.0 - lp * lp - mp * mp);
  const double aw = std::fabs(wproj);
  const double bx = 2.0 * ((aw * lp) / nn) * ((double)kp.o * kp.Lx);
  const double by = 2.0 * ((aw * mp) / nn) * ((double)kp.o * kp.Ly);
  const double B = bx > by ? bx : by;
  double nkd = 2.0 * std::ceil((kp.alpha * B) / 2.0) + 1.0;
  if (nkd > 1e6) nkd = 1e6;
  int nk = (int)nkd;
  if (capped && nk > kp.smax) nk = kp.smax;
  return nk;
}

namespace {

struct SortedSubset {
  std::vector<double> w;
  std::vector<long double> pre;  // pre[i] = sum of w[0..i)
  explicit SortedSubset(std::vector<double> v) : w(std::move(v)) {
    std::sort(w.begin(), w.end());
    pre.resize(w.size() + 1);
    pre[0] = 0.0L;
    for (size_t i = 0; i < w.size(); ++i) pre[i + 1] = pre[i] + (long double)w[i];
  }
};

std::vector<double> lloyd(const SortedSubset& S, int P) {
  const int64_t n = (int64_t)S.w.size();
  std::vector<double> c(P, 0.0);
  if (n == 0) return c;
  for (int p = 0; p < P; ++p) {
    int64_t i = (int64_t)std::floor((((double)p + 0.5) * (double)n) / (double)P);
    if (i > n - 1) i = n - 1;
    c[p] = S.w[i];
  }
  std::vector<int64_t> bound(P + 1, -1), nb(P + 1);
  for (int it = 0; it < 100; ++it) {
    nb[0] = 0;
    nb[P] = n;
    for (int p = 0; p < P - 1; ++p) {
      const double mid = 0.5 * (c[p] + c[p + 1]);
      // rows with w <= mid belong to bins <= p
      nb[p + 1] = std::upper_bound(S.w.begin(), S.w.end(), mid) - S.w.begin();
    }
    if (nb == bound) break;
    bound = nb;
    for (int p = 0; p < P; ++p) {
      const int64_t a = bound[p], b = bound[p + 1];
      if (b > a) c[p] = (double)((S.pre[b] - S.pre[a]) / (long double)(b - a));
    }
    std::sort(c.begin(), c.end());
  }
  std::sort(c.begin(), c.end());
  return c;
}

inline int bin_of(double w, const std::vector<double>& mids) {
  return (int)(std::lower_bound(mids.begin(), mids.end(), w) - mids.begin());
}

uint64_t splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

std::vector<double> kmeans_1d(std::vector<double> wsub, int P) {
  SortedSubset S(std::move(wsub));
  return lloyd(S, P);
}

int plan_channel(const double* w_all, int64_t M, const wf_image_shape& shape,
                 const wf_options& opt, uint64_t budget, PlanResult* out, std::string* err) {
  const int o = opt.oversample;
  const int nx = shape.nx, ny = shape.ny;
  const double cell = shape.cell_rad;
  KernelParams kp{};
  kp.Lx = nx * cell;
  kp.Ly = ny * cell;
  kp.oLx = o * kp.Lx;
  kp.oLy = o * kp.Ly;
  kp.alpha = opt.alpha;
  kp.smax = opt.smax;
  kp.o = o;
  kp.J = opt.J;
  // planning / clustering subset
  double f = opt.plan_fraction;
  if (M > 0) f = std::min(1.0, std::max(f, 20000.0 / (double)M));
  std::vector<double> wsub;
  if (f >= 1.0) {
    wsub.assign(w_all, w_all + M);
  } else {
    const uint64_t thr = (uint64_t)(f * 18446744073709551616.0);
    wsub.reserve((size_t)(f * M * 1.1) + 16);
    for (int64_t k = 0; k < M; ++k)
      if (splitmix64(opt.seed, (uint64_t)k) < thr) wsub.push_back(w_all[k]);
  }
  if (wsub.empty()) wsub.assign(w_all, w_all + std::min<int64_t>(M, 1));
  SortedSubset S(wsub);
  const int b_v = opt.store == WF_STORE_F32 ? 8 : 4;
  const double Kx = (double)o * nx, Ky = (double)o * ny;
  const double Np = Kx * Ky;
  const double grid_b = 8.0 * (2.0 * Np + ny * Kx + (double)nx * ny);
  const double scale_rows = (double)M / (double)S.w.size();
  // eq. 5 upper end of the search
  const double lmax = (nx / 2) * cell, mmax = (ny / 2) * cell;
  double wmin = w_all[0], wmax = w_all[0];
  for (int64_t k = 1; k < M; ++k) {
    wmin = std::min(wmin, w_all[k]);
    wmax = std::max(wmax, w_all[k]);
  }
  const double pw = 2.0 * M_PI * (wmax - wmin) * (1.0 - std::sqrt(1.0 - lmax * lmax - mmax * mmax));
  int Pmax = std::max(1, (int)std::ceil(pw));
  out->p_wsclean = Pmax;
  if (Pmax > 255) Pmax = 255;
  const double mstar = opt.budget_fraction * (double)budget;

  auto eval = [&](int P, double* K, double* ok, std::vector<double>* cents) {
    std::vector<double> c = lloyd(S, P);
    std::vector<double> mids(P > 1 ? P - 1 : 0);
    for (int p = 0; p + 1 < P; ++p) mids[p] = 0.5 * (c[p] + c[p + 1]);
    double sumT2 = 0.0;
    int64_t okc = 0;
    for (double w : S.w) {
      const int p = bin_of(w, mids);
      const int nk = nk_rule(w - c[p], kp, false);
      const double T = (double)(nk + opt.J - 1);
      sumT2 += T * T;
      if (nk <= opt.smax) ++okc;
    }
    *K = sumT2 * scale_rows;
    *ok = (double)okc / (double)S.w.size();
    if (cents) *cents = c;
  };

  if (opt.nbins > 0) {
    double K, ok;
    eval(opt.nbins, &K, &ok, &out->centroids);
    out->P = opt.nbins;
    out->p_star = opt.nbins;
    out->k_est = K;
    out->mem_model = b_v * K + 12.0 * M + grid_b;
    out->cost_model = 2.0 * (10.0 * Np * std::log2(std::sqrt(Np)) * opt.nbins + 6.0 * K);
    out->strategy = opt.strategy == WF_AUTO ? WF_PRECOMP_G : opt.strategy;
    return 0;
  }
  struct Row { int P; double K, ok, mem, cost; };
  std::vector<Row> tab;
  tab.reserve(Pmax);
  for (int P = 1; P <= Pmax; ++P) {
    double K, ok;
    eval(P, &K, &ok, nullptr);
    tab.push_back({P, K, ok, b_v * K + 12.0 * M + grid_b,
                   2.0 * (10.0 * Np * std::log2(std::sqrt(Np)) * P + 6.0 * K)});
  }
  int Pstar = 1;
  double cbest = tab[0].cost;
  for (const Row& r : tab)
    if (r.cost < cbest) {
      cbest = r.cost;
      Pstar = r.P;
    }
  out->p_star = Pstar;
  const Row* best = nullptr;
  for (const Row& r : tab) {
    if (r.mem <= mstar && r.ok >= 0.99) {
      if (!best) {
        best = &r;
        continue;
      }
      const int d0 = std::abs(best->P - Pstar), d1 = std::abs(r.P - Pstar);
      if (d1 < d0 || (d1 == d0 && r.cost < best->cost)) best = &r;
    }
  }
  if (best) {
    out->P = best->P;
    out->strategy = WF_PRECOMP_G;
    out->k_est = best->K;
    out->mem_model = best->mem;
    out->cost_model = best->cost;
    out->centroids = lloyd(S, best->P);
    return 0;
  }
  // no precomputed G fits: Fig. 2 branches (b) and (c)
  const double m_inf = b_v * (double)M * opt.J * opt.J + 12.0 * M + grid_b;
  int Pbar = Pmax;
  for (const Row& r : tab)
    if (r.mem <= 1.05 * m_inf) {
      Pbar = r.P;
      break;
    }
  out->P = Pbar;
  out->k_est = tab[Pbar - 1].K;
  out->mem_model = tab[Pbar - 1].mem;
  out->cost_model = tab[Pbar - 1].cost;
  out->strategy = WF_PRECOMP_H;
  out->centroids = lloyd(S, Pbar);
  // branch (b) when its exact size (known after the symbolic pass) fits, else (c)
  if (opt.strategy == WF_PRECOMP_G) {
    if (err) *err = "precomputed G does not fit the memory budget";
    return 1;
  }
  return 0;
}

void radix_sort_pairs(std::vector<uint64_t>& key, std::vector<int32_t>& idx, int lo_bit) {
  const size_t n = key.size();
  std::vector<uint64_t> k2(n);
  std::vector<int32_t> i2(n);
  for (int shift = lo_bit; shift < 64; shift += 8) {
    size_t cnt[257] = {0};
    for (size_t i = 0; i < n; ++i) ++cnt[((key[i] >> shift) & 0xff) + 1];
    bool trivial = false;
    for (int b = 0; b < 256; ++b)
      if (cnt[b + 1] == n) trivial = true;
    if (trivial) continue;
    for (int b = 0; b < 256; ++b) cnt[b + 1] += cnt[b];
    for (size_t i = 0; i < n; ++i) {
      const size_t d = cnt[(key[i] >> shift) & 0xff]++;
      k2[d] = key[i];
      i2[d] = idx[i];
    }
    key.swap(k2);
    idx.swap(i2);
  }
}

}  // namespace wf
