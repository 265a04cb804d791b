// C ABI of the library: cover construction (host), assembly of C and r on the
// device, and the bookkeeping around the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "cover.h"
#include "device_common.h"
#include "kernels.h"
#include "mc.h"
#include "runtime.h"

namespace pdd {

thread_local std::string g_last_error;

pdd_status fail(pdd_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

// ------------------------------------------------------ device block cache

namespace {

struct BlockCache {
  std::mutex mu;
  std::unordered_multimap<size_t, void*> free_blocks[64];   // per device, by rounded size
  size_t cached[64] = {};
  size_t cap[64] = {};
};

BlockCache& block_cache() {
  static BlockCache* c = new BlockCache();                   // lives until the process ends
  return *c;
}

size_t round_block(size_t bytes) {
  const size_t g = size_t(2) << 20;
  return (bytes + g - 1) / g * g;
}

// Frees the cached blocks of device d (caller holds the lock, d current).
size_t drop_cached(BlockCache& c, int d) {
  size_t n = 0;
  for (auto& kv : c.free_blocks[d]) {
    (void)hipFree(kv.second);
    n += kv.first;
  }
  c.free_blocks[d].clear();
  c.cached[d] = 0;
  return n;
}

}  // namespace

void* device_alloc(size_t bytes, int& device) {
  PDD_HIP(hipGetDevice(&device));
  const bool big = bytes >= kCacheMinBytes && device >= 0 && device < 64;
  const size_t size = big ? round_block(bytes) : bytes;
  BlockCache& c = block_cache();
  if (big) {
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.free_blocks[device].find(size);
    if (it != c.free_blocks[device].end()) {
      void* p = it->second;
      c.free_blocks[device].erase(it);
      c.cached[device] -= size;
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, size);
  if (e == hipErrorOutOfMemory && big) {       // give the cache back and try once more
    (void)hipGetLastError();
    {
      std::lock_guard<std::mutex> lk(c.mu);
      drop_cached(c, device);
    }
    e = hipMalloc(&p, size);
  }
  if (e != hipSuccess) throw HipError(e, "hipMalloc(" + std::to_string(bytes) + " bytes)");
  return p;
}

void device_free(void* p, size_t bytes, int device) {
  int cur = -1;
  const bool big = bytes >= kCacheMinBytes && device >= 0 && device < 64 &&
                   hipGetDevice(&cur) == hipSuccess && cur == device;
  if (!big) {
    (void)hipFree(p);
    return;
  }
  const size_t size = round_block(bytes);
  BlockCache& c = block_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  if (c.cap[device] == 0) {
    size_t fr = 0, total = 0;
    c.cap[device] = hipMemGetInfo(&fr, &total) == hipSuccess ? total / 2 : (size_t(16) << 30);
  }
  if (c.cached[device] + size > c.cap[device] || hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(p);
    return;
  }
  c.free_blocks[device].emplace(size, p);
  c.cached[device] += size;
}

size_t device_cache_release() {
  BlockCache& c = block_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return 0;
  size_t n = 0;
  for (int d = 0; d < 64; ++d) {
    if (c.free_blocks[d].empty()) continue;
    if (hipSetDevice(d) != hipSuccess) continue;
    n += drop_cached(c, d);
  }
  (void)hipSetDevice(cur);
  return n;
}

// ------------------------------------------------------------ device tables

static std::vector<double> cheb_points(int Nc) {
  std::vector<double> x(Nc + 1);
  for (int j = 0; j <= Nc; ++j) x[j] = std::cos(M_PI * j / Nc);
  return x;
}

// Chebyshev differentiation matrix on x_j = cos(j pi / Nc) (closed form, with
// differences x_i - x_j taken from the product-of-sines identity and the
// diagonal from the negative row sum).
static std::vector<double> cheb_diff(int Nc) {
  const int n1 = Nc + 1;
  std::vector<double> D((size_t)n1 * n1, 0.0);
  for (int i = 0; i < n1; ++i) {
    double rowsum = 0.0;
    for (int j = 0; j < n1; ++j) {
      if (i == j) continue;
      const double ci = (i == 0 || i == Nc) ? 2.0 : 1.0;
      const double cj = (j == 0 || j == Nc) ? 2.0 : 1.0;
      const double diff = 2.0 * std::sin((i + j) * M_PI / (2.0 * Nc)) * std::sin((j - i) * M_PI / (2.0 * Nc));
      const double v = (ci / cj) * (((i + j) & 1) ? -1.0 : 1.0) / diff;
      D[(size_t)i * n1 + j] = v;
      rowsum += v;
    }
    D[(size_t)i * n1 + i] = -rowsum;
  }
  return D;
}

// M-point periodic cardinal function sin(M x/2) cos(x/2) / (M sin(x/2)).
static double periodic_cardinal(int Mp, double x) {
  const double hx = 0.5 * x;
  const double s = std::sin(hx);
  if (std::fabs(s) < 1e-15) return 1.0;
  return std::sin(Mp * hx) * std::cos(hx) / (Mp * s);
}

void BucketData::build(int Nr_, int Nt_, int M_) {
  Nr = Nr_; Nt = Nt_; M = M_;
  Nc = 2 * Nr + 1;
  n = Nr * Nt;
  nrhs = M + 1;
  const int rhs_pad = ((nrhs + 15) / 16) * 16;
  ld = n + rhs_pad;
  const int n1 = Nc + 1;
  std::vector<double> x = cheb_points(Nc);
  std::vector<double> D = cheb_diff(Nc);
  std::vector<double> D2((size_t)n1 * n1, 0.0);
  for (int i = 0; i < n1; ++i)
    for (int k = 0; k < n1; ++k) {
      const double dik = D[(size_t)i * n1 + k];
      for (int j = 0; j < n1; ++j) D2[(size_t)i * n1 + j] += dik * D[(size_t)k * n1 + j];
    }
  std::vector<double> host;
  auto put = [&](const std::vector<double>& v) {
    size_t off = host.size();
    host.insert(host.end(), v.begin(), v.end());
    return off;
  };
  std::vector<double> Dr((size_t)Nr * n1), D2r((size_t)Nr * n1);
  for (int jr = 1; jr <= Nr; ++jr)
    for (int j = 0; j < n1; ++j) {
      Dr[(size_t)(jr - 1) * n1 + j] = D[(size_t)jr * n1 + j];
      D2r[(size_t)(jr - 1) * n1 + j] = D2[(size_t)jr * n1 + j];
    }
  const double h = 2.0 * M_PI / Nt;
  std::vector<double> d1(Nt), d2(Nt);
  d1[0] = 0.0;
  d2[0] = -M_PI * M_PI / (3.0 * h * h) - 1.0 / 6.0;
  for (int k = 1; k < Nt; ++k) {
    const double sgn = (k & 1) ? -1.0 : 1.0;
    const double sh = std::sin(0.5 * k * h);
    d1[k] = 0.5 * sgn * std::cos(0.5 * k * h) / sh;
    d2[k] = -0.5 * sgn / (sh * sh);
  }
  std::vector<double> H((size_t)Nt * M);
  for (int l = 0; l < Nt; ++l)
    for (int j = 0; j < M; ++j)
      H[(size_t)l * M + j] = periodic_cardinal(M, 2.0 * M_PI * l / Nt - 2.0 * M_PI * j / M);
  std::vector<double> bw(n1), cs(Nt), sn(Nt);
  for (int j = 0; j < n1; ++j) bw[j] = ((j & 1) ? -1.0 : 1.0) * ((j == 0 || j == Nc) ? 0.5 : 1.0);
  for (int l = 0; l < Nt; ++l) {
    cs[l] = std::cos(2.0 * M_PI * l / Nt);
    sn[l] = std::sin(2.0 * M_PI * l / Nt);
  }
  size_t oDr = put(Dr), oD2r = put(D2r), od1 = put(d1), od2 = put(d2), oH = put(H), ox = put(x),
         obw = put(bw), ocs = put(cs), osn = put(sn);
  tables.upload(host);
  const double* base = tables.ptr<double>();
  T.Nr = Nr; T.Nt = Nt; T.M = M; T.Nc = Nc; T.n = n; T.ld = ld; T.nrhs = nrhs;
  T.Dr = base + oDr; T.D2r = base + oD2r; T.d1t = base + od1; T.d2t = base + od2;
  T.H = base + oH; T.xr = base + ox; T.bw = base + obw; T.cs = base + ocs; T.sn = base + osn;
  host_H = H;
}

void DeviceCover::upload(const HostCover& Hc) {
  auto dbl = [](DevBuf& b, const std::vector<double>& v) { b.upload(v); };
  dbl(cx, Hc.cx); dbl(cy, Hc.cy); dbl(rad, Hc.r); dbl(arc0, Hc.arc0); dbl(arc1, Hc.arc1);
  dbl(rbf_c2, Hc.rbf_c2); dbl(kx, Hc.kx); dbl(ky, Hc.ky); dbl(ktheta, Hc.ktheta);
  knot_off.upload(Hc.knot_off); rowptr.upload(Hc.rowptr); cols.upload(Hc.cols);
  assigned.upload(Hc.assigned); float_ids.upload(Hc.float_ids); node_off.upload(Hc.node_off);
  fk_off.upload(Hc.fk_off); fk_ids.upload(Hc.fk_ids); perim_ids.upload(Hc.perim_ids);
  perim_pos.upload(Hc.perim_pos); mc_knots.upload(Hc.mc_knots); bnd_knots.upload(Hc.bnd_knots);
  pair_off.upload(Hc.pair_off); diag_pos.upload(Hc.diag_pos);
  pair_knot.upload(Hc.pair_knot); pair_seg.upload(Hc.pair_seg);
  have_transpose = false;
  have_blocked = false;
  buckets.clear();
  for (const Bucket& b : Hc.buckets) {
    auto bd = std::make_unique<BucketData>();
    bd->build(b.Nr, b.Nt, b.M);
    bd->fl.upload(b.fl);
    bd->count = (int32_t)b.fl.size();
    buckets.push_back(std::move(bd));
  }
  ready = true;
}

ChunkDesc DeviceCover::chunk(const BucketData& b, int32_t first, int32_t count) const {
  ChunkDesc C;
  C.count = count;
  C.fl = b.fl.ptr<int32_t>() + first;
  C.float_ids = float_ids.ptr<int32_t>();
  C.cx = cx.ptr<double>(); C.cy = cy.ptr<double>(); C.rad = rad.ptr<double>();
  C.node_off = node_off.ptr<int64_t>();
  C.fk_off = fk_off.ptr<int64_t>(); C.fk_ids = fk_ids.ptr<int32_t>();
  C.knot_off = knot_off.ptr<int64_t>();
  C.kx = kx.ptr<double>(); C.ky = ky.ptr<double>();
  C.rowptr = rowptr.ptr<int64_t>();
  return C;
}

static pdd_status to_dev_field(const pdd_field& f, DevField& d, const char* name) {
  std::memset(&d, 0, sizeof(d));
  d.kind = f.kind;
  d.n = f.n_terms;
  d.clip = f.clip_nonpos;
  d.base = f.base;
  if (f.kind < PDD_FIELD_CONST || f.kind > PDD_FIELD_EQ46)
    return fail(PDD_EINVAL, std::string("unknown field kind for ") + name);
  if (f.kind == PDD_FIELD_SINSUM || f.kind == PDD_FIELD_CPOLY_RE) {
    if (f.n_terms < 0 || f.n_terms > PDD_MAX_TERMS)
      return fail(PDD_EINVAL, std::string("too many terms in field ") + name);
    if (f.n_terms > 0 && (!f.a || !f.b || (f.kind == PDD_FIELD_SINSUM && (!f.c || !f.d))))
      return fail(PDD_EINVAL, std::string("missing term arrays in field ") + name);
    for (int q = 0; q < f.n_terms; ++q) {
      d.a[q] = f.a[q];
      d.b[q] = f.b[q];
      if (f.kind == PDD_FIELD_SINSUM) { d.c[q] = f.c[q]; d.d[q] = f.d[q]; }
    }
    if (f.kind == PDD_FIELD_SINSUM) {
      // integer wave numbers: a_q sin(2 pi (b_q x + c_q y) + d_q)
      //   = Im(a_q e^{i d_q} E^{b_q} F^{c_q}), E = e^{2 pi i x}, F = e^{2 pi i y}
      bool wave = true;
      for (int q = 0; q < f.n_terms; ++q)
        wave = wave && f.b[q] == std::nearbyint(f.b[q]) && f.c[q] == std::nearbyint(f.c[q]) &&
               std::fabs(f.b[q]) <= kWaveMax && std::fabs(f.c[q]) <= kWaveMax;
      d.wave = wave ? 1 : 0;
      for (int q = 0; wave && q < f.n_terms; ++q) {
        d.ix[q] = (int32_t)std::fabs(f.b[q]);
        d.iy[q] = (int32_t)std::fabs(f.c[q]);
        d.sx[q] = f.b[q] < 0 ? -1.0 : 1.0;
        d.sy[q] = f.c[q] < 0 ? -1.0 : 1.0;
        d.wr[q] = f.a[q] * std::cos(f.d[q]);
        d.wi[q] = f.a[q] * std::sin(f.d[q]);
      }
    }
  }
  return PDD_OK;
}

pdd_status make_dev_problem(const pdd_problem& p, DevProblem& D) {
  std::memset(&D, 0, sizeof(D));
  D.dom = p.domain;
  const pdd_field* fs[F_COUNT] = {&p.axx, &p.axy, &p.ayy, &p.bx, &p.by, &p.c, &p.f, &p.g, &p.u};
  const char* names[F_COUNT] = {"axx", "axy", "ayy", "bx", "by", "c", "f", "g", "u"};
  for (int t = 0; t < F_COUNT; ++t) {
    if (t != F_F && fs[t]->kind == PDD_FIELD_DERIVED_F)
      return fail(PDD_EINVAL, std::string("only f may be a derived field, not ") + names[t]);
    pdd_status s = to_dev_field(*fs[t], D.fld[t], names[t]);
    if (s != PDD_OK) return s;
  }
  bool allc = true;
  for (int t = 0; t < 7; ++t) allc = allc && fs[t]->kind == PDD_FIELD_CONST;
  D.const_coef = allc ? 1 : 0;
  auto wave_or_const = [&](int t) {
    return D.fld[t].kind == PDD_FIELD_CONST || (D.fld[t].kind == PDD_FIELD_SINSUM && D.fld[t].wave);
  };
  bool all = !allc;
  for (int t = 0; t < 6; ++t) all = all && wave_or_const(t);
  all = all && (wave_or_const(F_F) || (D.fld[F_F].kind == PDD_FIELD_DERIVED_F &&
                                       D.fld[F_U].kind == PDD_FIELD_SINSUM && D.fld[F_U].wave));
  D.wave_all = all ? 1 : 0;
  for (int t = 0; t < 7; ++t) D.k[t] = fs[t]->base;
  if (p.domain.kind == PDD_DOMAIN_DISK && (p.domain.n_holes < 0 || p.domain.n_holes > PDD_MAX_HOLES))
    return fail(PDD_EINVAL, "too many holes");
  return PDD_OK;
}

}  // namespace pdd

using namespace pdd;

// ------------------------------------------------------------------- C ABI

extern "C" {

int64_t pdd_release_cached_memory(void) { return (int64_t)pdd::device_cache_release(); }

const char* pdd_last_error(void) { return g_last_error.c_str(); }

pdd_status pdd_build_cover(const pdd_domain* domain, int32_t n_circles, const double* centres,
                           const double* radii, const int32_t* M, const int32_t* Ntheta,
                           const int32_t* Nr, const pdd_cover_opts* opts, pdd_cover* out) {
  if (!domain || !centres || !radii || !M || !Ntheta || !Nr || !out || n_circles <= 0)
    return fail(PDD_EINVAL, "pdd_build_cover: null argument or no circles");
  if (domain->kind != PDD_DOMAIN_BOX && domain->kind != PDD_DOMAIN_DISK)
    return fail(PDD_EINVAL, "pdd_build_cover: unknown domain kind");
  if (domain->kind == PDD_DOMAIN_DISK && (domain->n_holes < 0 || domain->n_holes > PDD_MAX_HOLES))
    return fail(PDD_EINVAL, "pdd_build_cover: too many holes");
  const int32_t rule = opts ? opts->rule : PDD_RULE_FLOAT_FIRST_MAX_DEPTH;
  if (rule < PDD_RULE_FLOAT_FIRST_MAX_DEPTH || rule > PDD_RULE_AVERAGED)
    return fail(PDD_EINVAL, "pdd_build_cover: unknown row rule");
  try {
    auto cv = std::make_unique<pdd_cover_s>();
    const double c2 = opts ? opts->rbf_c2 : 0.0;
    std::string err = build_host_cover(*domain, n_circles, centres, radii, M, Ntheta, Nr, rule, c2,
                                       cv->H);
    if (!err.empty()) return fail(PDD_ECOVER, "pdd_build_cover: " + err);
    for (int m = 0; m < n_circles; ++m) {
      if (cv->H.floating[m] && (cv->H.M[m] + 1 > 136 || (int64_t)cv->H.Nr[m] * cv->H.Nt[m] > 4096))
        return fail(PDD_EINVAL, "pdd_build_cover: M + 1 <= 136 and Nr Ntheta <= 4096 are supported");
    }
    if (cv->H.max_arc > 160) return fail(PDD_EINVAL, "pdd_build_cover: arcs of more than 160 knots");
    *out = cv.release();
    return PDD_OK;
  } catch (const std::bad_alloc&) {
    return fail(PDD_ENOMEM, "pdd_build_cover: out of host memory");
  } catch (const std::exception& e) {
    return fail(PDD_EINVAL, std::string("pdd_build_cover: ") + e.what());
  }
}

pdd_status pdd_cover_get_info(pdd_cover cover, pdd_cover_info* out) {
  if (!cover || !out) return fail(PDD_EINVAL, "pdd_cover_get_info: null argument");
  const HostCover& H = cover->H;
  std::memset(out, 0, sizeof(*out));
  out->N = H.N();
  out->nnz = H.rowptr.back();
  out->n_circles = H.nc;
  out->n_float = (int64_t)H.float_ids.size();
  out->n_perim = (int64_t)H.perim_ids.size();
  for (int32_t c : H.row_class) {
    if (c == ROW_SPECTRAL) ++out->n_spectral_rows;
    else if (c == ROW_MC) ++out->n_mc_rows;
    else ++out->n_boundary_rows;
  }
  out->sum_n = H.sum_n;
  out->sum_n2 = H.sum_n2;
  out->max_n = H.max_n;
  out->max_M = H.max_M;
  out->max_arc = H.max_arc;
  out->n_buckets = (int32_t)H.buckets.size();
  return PDD_OK;
}

pdd_status pdd_cover_knots(pdd_cover cover, double* xy, int32_t* row_class, int32_t* assigned,
                           int32_t* owner) {
  if (!cover) return fail(PDD_EINVAL, "pdd_cover_knots: null cover");
  const HostCover& H = cover->H;
  const int64_t N = H.N();
  for (int64_t i = 0; i < N; ++i) {
    if (xy) { xy[2 * i] = H.kx[i]; xy[2 * i + 1] = H.ky[i]; }
    if (row_class) row_class[i] = H.row_class[i];
    if (assigned) assigned[i] = H.assigned[i];
    if (owner) owner[i] = H.owner[i];
  }
  return PDD_OK;
}

pdd_status pdd_cover_pattern(pdd_cover cover, int64_t* rowptr, int32_t* cols) {
  if (!cover || !rowptr || !cols) return fail(PDD_EINVAL, "pdd_cover_pattern: null argument");
  std::copy(cover->H.rowptr.begin(), cover->H.rowptr.end(), rowptr);
  std::copy(cover->H.cols.begin(), cover->H.cols.end(), cols);
  return PDD_OK;
}

pdd_status pdd_cover_nodes(pdd_cover cover, double* xy, int64_t* node_off, int32_t* float_ids) {
  if (!cover) return fail(PDD_EINVAL, "pdd_cover_nodes: null cover");
  const HostCover& H = cover->H;
  for (size_t f = 0; f < H.float_ids.size(); ++f) {
    const int m = H.float_ids[f];
    const int Nr = H.Nr[m], Nt = H.Nt[m], Nc = 2 * Nr + 1;
    if (float_ids) float_ids[f] = m;
    if (xy) {
      for (int q = 0; q < Nr * Nt; ++q) {
        const int jr = q / Nt + 1, l = q % Nt;
        const double rr = H.r[m] * std::cos(M_PI * jr / Nc);
        const double th = 2.0 * M_PI * l / Nt;
        const int64_t node = H.node_off[f] + q;
        xy[2 * node] = H.cx[m] + rr * std::cos(th);
        xy[2 * node + 1] = H.cy[m] + rr * std::sin(th);
      }
    }
  }
  if (node_off) std::copy(H.node_off.begin(), H.node_off.end(), node_off);
  return PDD_OK;
}

void pdd_destroy_cover(pdd_cover cover) { delete cover; }

}  // extern "C"
