// Exact host-side stencil algebra: creation, composition C = B(A) and
// linear combination, all in rational arithmetic with 128-bit intermediates
// and explicit int64 overflow detection; plus the mapping of a stencil onto
// an instantiated kernel pattern.
#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>

#include "internal.hpp"

namespace sc {

namespace {

using i128 = __int128;
using Off = std::array<int32_t, 3>;

struct OffLess {
  bool operator()(const Off& a, const Off& b) const {
    if (a[2] != b[2]) return a[2] < b[2];
    if (a[1] != b[1]) return a[1] < b[1];
    return a[0] < b[0];
  }
};

i128 iabs128(i128 v) { return v < 0 ? -v : v; }

i128 gcd128(i128 a, i128 b) {
  a = iabs128(a);
  b = iabs128(b);
  while (b != 0) {
    const i128 t = a % b;
    a = b;
    b = t;
  }
  return a;
}

bool fits64(i128 v) { return v >= (i128)INT64_MIN && v <= (i128)INT64_MAX; }

bool add_ok(i128 a, i128 b, i128* out) { return !__builtin_add_overflow(a, b, out); }
bool mul_ok(i128 a, i128 b, i128* out) { return !__builtin_mul_overflow(a, b, out); }

// Build a canonical stencil from accumulated 128-bit numerators over `den`.
sc_status finish(int dim, int hpow, std::map<Off, i128, OffLess>& acc, i128 den, sc_stencil** out) {
  if (den == 0) {
    set_error("zero denominator");
    return SC_EINVAL;
  }
  if (den < 0) {
    den = -den;
    for (auto& kv : acc) kv.second = -kv.second;
  }
  i128 g = den;
  for (auto& kv : acc)
    if (kv.second != 0) g = gcd128(g, kv.second);
  if (g == 0) g = 1;
  auto* s = new sc_stencil();
  s->dim = dim;
  s->hpow = hpow;
  const i128 d = den / g;
  if (!fits64(d)) {
    delete s;
    set_error("denominator exceeds int64");
    return SC_EOVERFLOW;
  }
  s->den = (int64_t)d;
  for (auto& kv : acc) {
    if (kv.second == 0) continue;
    const i128 v = kv.second / g;
    if (!fits64(v)) {
      delete s;
      set_error("numerator exceeds int64");
      return SC_EOVERFLOW;
    }
    s->off.push_back(kv.first);
    s->num.push_back((int64_t)v);
  }
  if (s->off.empty()) {
    // the zero operator: keep one explicit zero tap at the origin so the
    // stencil still has a dimension and radius 0
    s->off.push_back(Off{0, 0, 0});
    s->num.push_back(0);
    s->den = 1;
  }
  *out = s;
  return SC_OK;
}

}  // namespace

sc_status stencil_create(int32_t dim, int32_t npts, const int32_t* offsets, const int64_t* num,
                         int64_t den, int32_t hpow, sc_stencil** out) {
  if (!out || !offsets || !num) {
    set_error("NULL argument");
    return SC_EINVAL;
  }
  *out = nullptr;
  if (dim < 1 || dim > 3 || npts < 1 || den == 0) {
    set_error("invalid stencil: dim=%d npts=%d den=%lld", dim, npts, (long long)den);
    return SC_EINVAL;
  }
  std::map<Off, i128, OffLess> acc;
  for (int t = 0; t < npts; ++t) {
    Off o{offsets[3 * t], offsets[3 * t + 1], offsets[3 * t + 2]};
    for (int d = 0; d < 3; ++d) {
      if (o[d] < -64 || o[d] > 64 || (d >= dim && o[d] != 0)) {
        set_error("offset component %d of tap %d out of range", d, t);
        return SC_EINVAL;
      }
    }
    i128 v;
    if (!add_ok(acc[o], (i128)num[t], &v)) {
      set_error("overflow while merging taps");
      return SC_EOVERFLOW;
    }
    acc[o] = v;
  }
  return finish(dim, hpow, acc, (i128)den, out);
}

// C = B(A): C[u + v] = sum a_u b_v over a common denominator den_a den_b.
sc_status compose(const sc_stencil* a, const sc_stencil* b, sc_stencil** out) {
  if (!a || !b || !out) {
    set_error("NULL argument");
    return SC_EINVAL;
  }
  *out = nullptr;
  if (a->dim != b->dim) {
    set_error("dimension mismatch (%d vs %d)", a->dim, b->dim);
    return SC_EINVAL;
  }
  std::map<Off, i128, OffLess> acc;
  for (size_t i = 0; i < a->off.size(); ++i) {
    for (size_t j = 0; j < b->off.size(); ++j) {
      Off o{a->off[i][0] + b->off[j][0], a->off[i][1] + b->off[j][1], a->off[i][2] + b->off[j][2]};
      if (std::abs(o[0]) > 64 || std::abs(o[1]) > 64 || std::abs(o[2]) > 64) {
        set_error("composed offset out of range");
        return SC_EINVAL;
      }
      i128 prod, sum;
      if (!mul_ok((i128)a->num[i], (i128)b->num[j], &prod) || !add_ok(acc[o], prod, &sum)) {
        set_error("overflow in composition");
        return SC_EOVERFLOW;
      }
      acc[o] = sum;
    }
  }
  i128 den;
  if (!mul_ok((i128)a->den, (i128)b->den, &den)) {
    set_error("overflow in composed denominator");
    return SC_EOVERFLOW;
  }
  return finish(a->dim, a->hpow + b->hpow, acc, den, out);
}

// sum_k (cnum_k / cden_k) h^{chpow_k} S_k
sc_status lincomb(int32_t n, const sc_stencil* const* terms, const int64_t* cnum, const int64_t* cden,
                  const int32_t* chpow, sc_stencil** out) {
  if (!terms || !cnum || !cden || !chpow || !out || n < 1) {
    set_error("invalid linear combination arguments");
    return SC_EINVAL;
  }
  *out = nullptr;
  const int dim = terms[0] ? terms[0]->dim : 0;
  const int p = terms[0] ? terms[0]->hpow - chpow[0] : 0;
  // common denominator D = lcm_k(cden_k * den_k)
  i128 D = 1;
  for (int k = 0; k < n; ++k) {
    if (!terms[k] || terms[k]->dim != dim || terms[k]->hpow - chpow[k] != p || cden[k] == 0) {
      set_error("term %d is incompatible", k);
      return SC_EINVAL;
    }
    i128 dk;
    if (!mul_ok((i128)cden[k], (i128)terms[k]->den, &dk)) {
      set_error("overflow in linear combination");
      return SC_EOVERFLOW;
    }
    dk = iabs128(dk);
    const i128 g = gcd128(D, dk);
    i128 l;
    if (!mul_ok(D / g, dk, &l)) {
      set_error("overflow in linear combination");
      return SC_EOVERFLOW;
    }
    D = l;
  }
  std::map<Off, i128, OffLess> acc;
  for (int k = 0; k < n; ++k) {
    const sc_stencil* s = terms[k];
    i128 dk = (i128)cden[k] * (i128)s->den;
    const i128 factor = D / iabs128(dk) * (dk < 0 ? -1 : 1);
    for (size_t t = 0; t < s->off.size(); ++t) {
      i128 v, w, sum;
      if (!mul_ok((i128)cnum[k], (i128)s->num[t], &v) || !mul_ok(v, factor, &w) ||
          !add_ok(acc[s->off[t]], w, &sum)) {
        set_error("overflow in linear combination");
        return SC_EOVERFLOW;
      }
      acc[s->off[t]] = sum;
    }
  }
  return finish(dim, p, acc, D, out);
}

// ------------------------------------------------------------ patterns
namespace {

struct Cand {
  int pat, R;
};
// Instantiated kernels per dimension (see dispatch.hip); ordering does not
// matter, the cheapest container is chosen.
const Cand kCand2[] = {{PAT_CROSS, 1}, {PAT_CROSS, 2}, {PAT_DIAMOND, 2}, {PAT_CROSSBOX, 4},
                       {PAT_BOX, 1},   {PAT_BOX, 2},   {PAT_BOX, 3},     {PAT_BOX, 4}};
const Cand kCand3[] = {{PAT_CROSS, 1}, {PAT_CROSS, 2}, {PAT_DIAMOND, 2}, {PAT_BOX, 1}, {PAT_BOX, 2}};

}  // namespace

sc_status make_kstencil(int dim, const std::vector<std::array<int32_t, 3>>& off,
                        const std::vector<long double>& w, KStencil* out) {
  if (dim != 2 && dim != 3) {
    set_error("only 2D and 3D grids are supported (dim=%d)", dim);
    return SC_EUNSUPPORTED;
  }
  const Cand* cands = dim == 2 ? kCand2 : kCand3;
  const int ncand = dim == 2 ? (int)(sizeof(kCand2) / sizeof(Cand)) : (int)(sizeof(kCand3) / sizeof(Cand));
  // a kernel reads every tap of its pattern (zero weights included), so the
  // pattern's radius must be the stencil's own: callers size rings by it
  int radius = 1;  // a lone centre tap still runs a radius-1 kernel
  for (const auto& o : off)
    for (int a = 0; a < 3; ++a) radius = std::max(radius, std::abs((int)o[a]));
  int best = -1, best_taps = 1 << 30;
  for (int c = 0; c < ncand; ++c) {
    if (cands[c].R != radius) continue;
    bool ok = true;
    for (const auto& o : off) {
      if (!in_pattern(cands[c].pat, cands[c].R, o[0], o[1], dim == 3 ? o[2] : 0) || (dim == 2 && o[2] != 0)) {
        ok = false;
        break;
      }
    }
    const int nt = num_taps(cands[c].pat, cands[c].R, dim);
    if (ok && nt < best_taps) {
      best = c;
      best_taps = nt;
    }
  }
  if (best < 0) {
    set_error("no kernel for this stencil support in %dD (max radius %d)", dim, dim == 2 ? 4 : 2);
    return SC_EUNSUPPORTED;
  }
  KStencil ks;
  ks.dim = dim;
  ks.pat = cands[best].pat;
  ks.R = cands[best].R;
  ks.ntaps = best_taps;
  for (size_t t = 0; t < off.size(); ++t) {
    const int idx = tap_index(ks.pat, ks.R, dim, off[t][0], off[t][1], dim == 3 ? off[t][2] : 0);
    ks.w[idx] = (double)w[t];
  }
  // mirror symmetry: negating any one offset component keeps the weight
  ks.sym = true;
  const int zr = dim == 3 ? ks.R : 0;
  for (int z = -zr; z <= zr && ks.sym; ++z)
    for (int y = -ks.R; y <= ks.R && ks.sym; ++y)
      for (int x = -ks.R; x <= ks.R && ks.sym; ++x) {
        if (!in_pattern(ks.pat, ks.R, x, y, z)) continue;
        const double v = ks.w[tap_index(ks.pat, ks.R, dim, x, y, z)];
        if (v != ks.w[tap_index(ks.pat, ks.R, dim, -x, y, z)] || v != ks.w[tap_index(ks.pat, ks.R, dim, x, -y, z)] ||
            v != ks.w[tap_index(ks.pat, ks.R, dim, x, y, -z)])
          ks.sym = false;
      }
  *out = ks;
  return SC_OK;
}

KStencil to_box(const KStencil& ks) {
  KStencil b;
  b.dim = ks.dim;
  b.pat = PAT_BOX;
  b.R = ks.R;
  b.ntaps = num_taps(PAT_BOX, ks.R, ks.dim);
  b.sym = false;
  const int zr = ks.dim == 3 ? ks.R : 0;
  for (int z = -zr; z <= zr; ++z)
    for (int y = -ks.R; y <= ks.R; ++y)
      for (int x = -ks.R; x <= ks.R; ++x)
        if (in_pattern(ks.pat, ks.R, x, y, z))
          b.w[tap_index(PAT_BOX, ks.R, ks.dim, x, y, z)] = ks.w[tap_index(ks.pat, ks.R, ks.dim, x, y, z)];
  return b;
}

TapTable tap_table(const KStencil& ks) {
  TapTable t;
  const int zr = ks.dim == 3 ? ks.R : 0;
  for (int z = -zr; z <= zr; ++z)
    for (int y = -ks.R; y <= ks.R; ++y)
      for (int x = -ks.R; x <= ks.R; ++x) {
        if (!in_pattern(ks.pat, ks.R, x, y, z)) continue;
        const double w = ks.w[tap_index(ks.pat, ks.R, ks.dim, x, y, z)];
        if (w == 0.0 || t.n >= kMaxTaps) continue;
        t.off[t.n][0] = x;
        t.off[t.n][1] = y;
        t.off[t.n][2] = z;
        t.w[t.n] = w;
        ++t.n;
      }
  return t;
}

sc_status make_kstencil(const sc_stencil* s, double h, KStencil* out) {
  if (!s || !(h > 0.0) || !std::isfinite(h)) {
    set_error("invalid stencil or grid spacing");
    return SC_EINVAL;
  }
  // weight = num / (den h^p), evaluated in extended precision and rounded
  // once to double
  long double hp = 1.0L;
  for (int i = 0; i < std::abs(s->hpow); ++i) hp *= (long double)h;
  if (s->hpow < 0) hp = 1.0L / hp;
  std::vector<long double> w(s->num.size());
  for (size_t t = 0; t < s->num.size(); ++t) w[t] = (long double)s->num[t] / ((long double)s->den * hp);
  return make_kstencil(s->dim, s->off, w, out);
}

}  // namespace sc
