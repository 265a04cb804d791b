// Host-side cover geometry: subdomain classification, interface arcs, knots,
// stencils and the row choice (Section 2.1, eqs. 4-12; Section 3.2).
//
// Readings: a circle is floating when its closed disk lies in Omega; otherwise
// its interface is the single arc of the circle inside closure(Omega).  Knots
// sit at the global angles 2 pi j / M (floating: all of them; arcs: those
// inside the arc at least dtheta/4 from its ends, plus the two junction knots
// on the boundary).  A knot's row comes from the deepest floating circle that
// contains it strictly (depth r - |x - c| > 1e-9 r), else from the deepest
// perimeter circle; a later circle wins only if deeper by more than 1e-12 r.
#include "cover.h"

#include <algorithm>
#include <cmath>
#include <unordered_map>

namespace pdd {

namespace {

constexpr double kTwoPi = 2.0 * M_PI;

double wrap_2pi(double a) {
  double w = std::fmod(a, kTwoPi);
  if (w < 0.0) w += kTwoPi;
  return w;
}

bool inside(const pdd_domain& d, double x, double y) { return signed_distance(d, x, y) > 0.0; }

// Angles at which the circle (cx, cy, r) meets the boundary of the domain.
std::vector<double> crossings(const pdd_domain& d, double cx, double cy, double r) {
  std::vector<double> a;
  if (d.kind == PDD_DOMAIN_BOX) {
    const double xs[2] = {d.x0, d.x1};
    for (double xv : xs) {
      double t = (xv - cx) / r;
      if (std::fabs(t) < 1.0) {
        double ang = std::acos(t);
        a.push_back(ang);
        a.push_back(-ang);
      }
    }
    const double ys[2] = {d.y0, d.y1};
    for (double yv : ys) {
      double t = (yv - cy) / r;
      if (std::fabs(t) < 1.0) {
        double ang = std::asin(t);
        a.push_back(ang);
        a.push_back(M_PI - ang);
      }
    }
  } else {
    double bc[1 + PDD_MAX_HOLES][3];
    int nb = 0;
    bc[nb][0] = d.cx; bc[nb][1] = d.cy; bc[nb][2] = d.R; ++nb;
    for (int h = 0; h < d.n_holes; ++h, ++nb)
      for (int t = 0; t < 3; ++t) bc[nb][t] = d.holes[h][t];
    for (int b = 0; b < nb; ++b) {
      double dx = bc[b][0] - cx, dy = bc[b][1] - cy, br = bc[b][2];
      double dist = std::sqrt(dx * dx + dy * dy);
      if (std::fabs(r - br) < dist && dist < r + br) {
        double alpha = std::atan2(dy, dx);
        double beta = std::acos((r * r + dist * dist - br * br) / (2.0 * r * dist));
        a.push_back(alpha + beta);
        a.push_back(alpha - beta);
      }
    }
  }
  for (double& v : a) v = wrap_2pi(v);
  std::sort(a.begin(), a.end());
  return a;
}

// Single interface arc (theta_min, theta_max) of a perimeter circle (eqs. 8, 11).
std::string arc_of(const pdd_domain& d, double cx, double cy, double r, double& t0, double& t1) {
  std::vector<double> raw = crossings(d, cx, cy, r);
  std::vector<double> u;
  for (double v : raw)
    if (u.empty() || v - u.back() > 1e-14) u.push_back(v);
  if (u.size() > 1 && u.front() + kTwoPi - u.back() <= 1e-14) u.pop_back();
  if (u.empty()) return "a non-floating circle does not cross the boundary";
  const size_t k = u.size();
  std::vector<char> in(k);
  for (size_t t = 0; t < k; ++t) {
    double a0 = u[t];
    double a1 = (t + 1 == k) ? u[0] + kTwoPi : u[t + 1];
    double mid = 0.5 * (a0 + a1);
    in[t] = inside(d, cx + r * std::cos(mid), cy + r * std::sin(mid));
  }
  size_t n_in = 0, start = 0, n_start = 0;
  for (size_t t = 0; t < k; ++t) {
    n_in += in[t];
    if (in[t] && !in[(t + k - 1) % k]) { start = t; ++n_start; }
  }
  if (n_in == k) return "a circle touches the boundary without crossing it";
  if (n_in == 0) return "a circle's interface lies outside the domain";
  if (n_start != 1) return "a perimeter interface has more than one arc";
  size_t e = start;
  while (in[(e + 1) % k]) ++e;
  t0 = u[start];
  t1 = u[(e + 1) % k];
  if (t1 <= t0) t1 += kTwoPi;
  return "";
}

}  // namespace

double signed_distance(const pdd_domain& d, double x, double y) {
  if (d.kind == PDD_DOMAIN_BOX)
    return std::min(std::min(x - d.x0, d.x1 - x), std::min(y - d.y0, d.y1 - y));
  double s = d.R - std::sqrt((x - d.cx) * (x - d.cx) + (y - d.cy) * (y - d.cy));
  for (int h = 0; h < d.n_holes; ++h) {
    double hx = d.holes[h][0], hy = d.holes[h][1], hr = d.holes[h][2];
    s = std::min(s, std::sqrt((x - hx) * (x - hx) + (y - hy) * (y - hy)) - hr);
  }
  return s;
}

// Floating and perimeter circle tables, the rows each floating circle
// evaluates, the Monte Carlo and boundary knots, and the size buckets.
static void finish_tables(HostCover& C) {
  const int n = C.nc;
  const int64_t N = C.N();
  C.float_pos.assign(n, -1);
  C.perim_pos.assign(n, -1);
  // floating-circle tables
  C.node_off.push_back(0);
  for (int m = 0; m < n; ++m) {
    if (C.floating[m]) {
      C.float_pos[m] = (int32_t)C.float_ids.size();
      C.float_ids.push_back(m);
      int64_t nn = (int64_t)C.Nr[m] * C.Nt[m];
      C.node_off.push_back(C.node_off.back() + nn);
      C.sum_n += nn;
      C.sum_n2 += nn * nn;
      C.max_n = std::max<int32_t>(C.max_n, (int32_t)nn);
    } else {
      C.perim_pos[m] = (int32_t)C.perim_ids.size();
      C.perim_ids.push_back(m);
      C.max_arc = std::max<int32_t>(C.max_arc, (int32_t)(C.knot_off[m + 1] - C.knot_off[m]));
    }
    C.max_M = std::max(C.max_M, C.M[m]);
  }
  const size_t nf = C.float_ids.size();
  std::vector<int64_t> cnt(nf + 1, 0);
  for (int64_t i = 0; i < N; ++i)
    if (C.row_class[i] == ROW_SPECTRAL) ++cnt[C.float_pos[C.assigned[i]] + 1];
  C.fk_off.assign(nf + 1, 0);
  for (size_t f = 0; f < nf; ++f) C.fk_off[f + 1] = C.fk_off[f] + cnt[f + 1];
  C.fk_ids.resize(C.fk_off[nf]);
  std::vector<int64_t> fill(C.fk_off.begin(), C.fk_off.end() - 1);
  for (int64_t i = 0; i < N; ++i)
    if (C.row_class[i] == ROW_SPECTRAL) C.fk_ids[fill[C.float_pos[C.assigned[i]]]++] = (int32_t)i;
  // Monte Carlo knots grouped by circle, boundary knots
  std::vector<std::vector<int32_t>> per(C.perim_ids.size());
  for (int64_t i = 0; i < N; ++i) {
    if (C.row_class[i] == ROW_MC) per[C.perim_pos[C.assigned[i]]].push_back((int32_t)i);
    if (C.row_class[i] == ROW_BOUNDARY) C.bnd_knots.push_back((int32_t)i);
  }
  for (auto& v : per) C.mc_knots.insert(C.mc_knots.end(), v.begin(), v.end());
  // size buckets of floating circles
  for (size_t f = 0; f < nf; ++f) {
    int m = C.float_ids[f];
    Bucket* b = nullptr;
    for (auto& bb : C.buckets)
      if (bb.Nr == C.Nr[m] && bb.Nt == C.Nt[m] && bb.M == C.M[m]) b = &bb;
    if (!b) {
      C.buckets.push_back({C.Nr[m], C.Nt[m], C.M[m], {}});
      b = &C.buckets.back();
    }
    b->fl.push_back((int32_t)f);
  }
}

std::string build_host_cover(const pdd_domain& dom, int32_t n, const double* centres,
                             const double* radii, const int32_t* Mv, const int32_t* Ntv,
                             const int32_t* Nrv, int32_t rule, double rbf_c2, HostCover& C) {
  C = HostCover();
  if (rule < PDD_RULE_FLOAT_FIRST_MAX_DEPTH || rule > PDD_RULE_AVERAGED) return "unknown row rule";
  C.dom = dom;
  C.nc = n;
  C.cx.resize(n); C.cy.resize(n); C.r.resize(n);
  C.M.assign(Mv, Mv + n); C.Nt.assign(Ntv, Ntv + n); C.Nr.assign(Nrv, Nrv + n);
  C.floating.assign(n, 0);
  C.arc0.assign(n, 0.0); C.arc1.assign(n, 0.0); C.rbf_c2.assign(n, 0.0);
  C.float_pos.assign(n, -1);
  C.perim_pos.assign(n, -1);
  C.knot_off.push_back(0);
  for (int m = 0; m < n; ++m) {
    C.cx[m] = centres[2 * m];
    C.cy[m] = centres[2 * m + 1];
    C.r[m] = radii[m];
    if (!(C.r[m] > 0.0) || C.M[m] < 2) return "radii must be positive and M >= 2";
  }
  // classification and knots, circle by circle
  for (int m = 0; m < n; ++m) {
    const double cx = C.cx[m], cy = C.cy[m], r = C.r[m];
    const int Mm = C.M[m];
    const double sd = signed_distance(dom, cx, cy);
    if (sd - r > 1e-12 * r) {
      if (Mm % 2 || C.Nt[m] % 2 || C.Nt[m] < 2 || C.Nr[m] < 1)
        return "floating circles need even M and Ntheta and Nr >= 1";
      C.floating[m] = 1;
      for (int j = 0; j < Mm; ++j) {
        double a = kTwoPi * j / Mm;
        C.kx.push_back(cx + r * std::cos(a));
        C.ky.push_back(cy + r * std::sin(a));
        C.ktheta.push_back(a);
        C.owner.push_back(m);
        C.boundary.push_back(0);
      }
    } else {
      double t0 = 0, t1 = 0;
      std::string err = arc_of(dom, cx, cy, r, t0, t1);
      if (!err.empty()) return err + " (circle " + std::to_string(m) + ")";
      C.arc0[m] = t0;
      C.arc1[m] = t1;
      const double span = t1 - t0, dth = kTwoPi / Mm;
      struct K { double loc, c, s; };
      std::vector<K> grid;
      for (int j = 0; j < Mm; ++j) {
        double a = kTwoPi * j / Mm;
        double off = wrap_2pi(a - t0);
        if (off > 0.25 * dth && off < span - 0.25 * dth)
          grid.push_back({t0 + off, std::cos(a), std::sin(a)});
      }
      std::sort(grid.begin(), grid.end(), [](const K& p, const K& q) { return p.loc < q.loc; });
      auto push = [&](double loc, double c, double s, bool bnd) {
        C.kx.push_back(cx + r * c);
        C.ky.push_back(cy + r * s);
        C.ktheta.push_back(loc);
        C.owner.push_back(m);
        C.boundary.push_back(bnd ? 1 : 0);
      };
      push(t0, std::cos(t0), std::sin(t0), true);
      for (const K& g : grid) push(g.loc, g.c, g.s, false);
      push(t1, std::cos(t1), std::sin(t1), true);
      C.rbf_c2[m] = rbf_c2 > 0.0 ? rbf_c2 : 1.5 * (44.0 / Mm) * (44.0 / Mm);
    }
    C.knot_off.push_back((int64_t)C.kx.size());
  }
  const int64_t N = C.N();

  // spatial hash of circle centres for candidate search
  double rmax = 0.0, xmin = 1e300, ymin = 1e300;
  for (int m = 0; m < n; ++m) {
    rmax = std::max(rmax, C.r[m]);
    xmin = std::min(xmin, C.cx[m]);
    ymin = std::min(ymin, C.cy[m]);
  }
  const double cell = rmax * (1.0 + 1e-9);
  auto key = [&](int64_t ix, int64_t iy) { return (ix << 32) ^ (iy & 0xffffffffLL); };
  std::unordered_map<int64_t, std::vector<int32_t>> hash;
  for (int m = 0; m < n; ++m) {
    int64_t ix = (int64_t)std::floor((C.cx[m] - xmin) / cell);
    int64_t iy = (int64_t)std::floor((C.cy[m] - ymin) / cell);
    hash[key(ix, iy)].push_back(m);
  }

  C.assigned.assign(N, -1);
  C.row_class.assign(N, ROW_BOUNDARY);
  const bool averaged = rule == PDD_RULE_AVERAGED;
  std::vector<std::vector<int32_t>> cont(averaged ? N : 0);
  std::vector<int32_t> cand;
  for (int64_t i = 0; i < N; ++i) {
    if (C.boundary[i]) continue;
    const double x = C.kx[i], y = C.ky[i];
    int64_t ix = (int64_t)std::floor((x - xmin) / cell);
    int64_t iy = (int64_t)std::floor((y - ymin) / cell);
    cand.clear();
    for (int64_t a = ix - 1; a <= ix + 1; ++a)
      for (int64_t b = iy - 1; b <= iy + 1; ++b) {
        auto it = hash.find(key(a, b));
        if (it != hash.end()) cand.insert(cand.end(), it->second.begin(), it->second.end());
      }
    std::sort(cand.begin(), cand.end());
    int32_t best[2] = {-1, -1};      // [0] floating (or any, MAX_DEPTH), [1] perimeter
    double bestd[2] = {0.0, 0.0};
    for (int32_t m : cand) {
      if (m == C.owner[i]) continue;
      double dx = x - C.cx[m], dy = y - C.cy[m];
      double depth = C.r[m] - std::sqrt(dx * dx + dy * dy);
      if (depth <= 1e-9 * C.r[m]) continue;
      if (averaged) cont[i].push_back(m);
      int slot = (rule == PDD_RULE_MAX_DEPTH) ? 0 : (C.floating[m] ? 0 : 1);
      if (best[slot] < 0 || depth > bestd[slot] + 1e-12 * C.r[m]) {
        best[slot] = m;
        bestd[slot] = depth;
      }
    }
    int32_t m = best[0] >= 0 ? best[0] : best[1];
    if (m < 0) return "knot " + std::to_string(i) + " is not interior to any other subdomain";
    C.assigned[i] = m;
    C.row_class[i] = C.floating[m] ? ROW_SPECTRAL : ROW_MC;
  }

  if (averaged) {
    // CSR pattern: diagonal plus the stencils of all containing circles
    // (contiguous knot ranges in circle order; x_i is on none of them)
    C.rowptr.assign(N + 1, 0);
    for (int64_t i = 0; i < N; ++i) {
      int64_t len = 1;
      if (C.row_class[i] != ROW_BOUNDARY)
        for (int32_t m : cont[i]) len += C.knot_off[m + 1] - C.knot_off[m];
      C.rowptr[i + 1] = C.rowptr[i] + len;
    }
    C.cols.resize(C.rowptr[N]);
    C.diag_pos.assign(N, 0);
    for (int64_t i = 0; i < N; ++i) {
      int64_t p = C.rowptr[i];
      bool placed = false;
      if (C.row_class[i] != ROW_BOUNDARY)
        for (int32_t m : cont[i]) {
          if (!placed && i < C.knot_off[m]) {
            C.diag_pos[i] = p;
            C.cols[p++] = (int32_t)i;
            placed = true;
          }
          for (int64_t j = C.knot_off[m]; j < C.knot_off[m + 1]; ++j) C.cols[p++] = (int32_t)j;
        }
      if (!placed) {
        C.diag_pos[i] = p;
        C.cols[p++] = (int32_t)i;
      }
    }
  } else {
    // CSR pattern: diagonal plus the stencil of the chosen circle, columns sorted
    C.rowptr.assign(N + 1, 0);
    for (int64_t i = 0; i < N; ++i) {
      int64_t len = 1;
      if (C.row_class[i] != ROW_BOUNDARY) {
        int m = C.assigned[i];
        len += C.knot_off[m + 1] - C.knot_off[m];
      }
      C.rowptr[i + 1] = C.rowptr[i] + len;
    }
    C.cols.resize(C.rowptr[N]);
    for (int64_t i = 0; i < N; ++i) {
      int64_t p = C.rowptr[i];
      if (C.row_class[i] == ROW_BOUNDARY) {
        C.cols[p] = (int32_t)i;
        continue;
      }
      int m = C.assigned[i];
      int64_t lo = C.knot_off[m], hi = C.knot_off[m + 1];
      if (i < lo) C.cols[p++] = (int32_t)i;
      for (int64_t j = lo; j < hi; ++j) C.cols[p++] = (int32_t)j;
      if (i > lo) C.cols[p++] = (int32_t)i;   // i is never inside [lo, hi)
    }
  }

  finish_tables(C);
  if (averaged) {
    // the pairs (knot i, circle m containing x_i), in knot then circle order
    auto P = std::make_unique<HostCover>();
    HostCover& Q = *P;
    Q.dom = C.dom; Q.nc = C.nc;
    Q.cx = C.cx; Q.cy = C.cy; Q.r = C.r; Q.arc0 = C.arc0; Q.arc1 = C.arc1; Q.rbf_c2 = C.rbf_c2;
    Q.M = C.M; Q.Nt = C.Nt; Q.Nr = C.Nr; Q.floating = C.floating;
    Q.knot_off = C.knot_off; Q.ktheta = C.ktheta;
    C.pair_off.assign(N + 1, 0);
    for (int64_t i = 0; i < N; ++i) {
      if (C.row_class[i] != ROW_BOUNDARY)
        for (int32_t m : cont[i]) {
          Q.kx.push_back(C.kx[i]);
          Q.ky.push_back(C.ky[i]);
          Q.owner.push_back(C.owner[i]);
          Q.boundary.push_back(0);
          Q.assigned.push_back(m);
          Q.row_class.push_back(C.floating[m] ? ROW_SPECTRAL : ROW_MC);
          Q.pair_knot.push_back((int32_t)i);
          // circle m's entries in row i: after the columns of row i below knot_off[m]
          int64_t pos = C.rowptr[i];
          while (pos < C.rowptr[i + 1] && C.cols[pos] < C.knot_off[m]) ++pos;
          Q.pair_seg.push_back(pos);
        }
      C.pair_off[i + 1] = (int64_t)Q.kx.size();
    }
    // pair rows as the kernels lay a row out: the diagonal slot, then the
    // stencil, the diagonal slot first when the row index is below the stencil
    const int64_t np = Q.N();
    Q.rowptr.assign(np + 1, 0);
    for (int64_t q = 0; q < np; ++q) {
      const int m = Q.assigned[q];
      Q.rowptr[q + 1] = Q.rowptr[q] + 1 + (C.knot_off[m + 1] - C.knot_off[m]);
    }
    Q.cols.resize(Q.rowptr[np]);
    for (int64_t q = 0; q < np; ++q) {
      const int m = Q.assigned[q];
      int64_t p = Q.rowptr[q];
      const int64_t lo = C.knot_off[m], hi = C.knot_off[m + 1];
      if (q < lo) Q.cols[p++] = (int32_t)Q.pair_knot[q];
      for (int64_t j = lo; j < hi; ++j) Q.cols[p++] = (int32_t)j;
      if (q >= lo) Q.cols[p++] = (int32_t)Q.pair_knot[q];
    }
    finish_tables(Q);
    C.pairs = std::move(P);
  }
  return "";
}

}  // namespace pdd
