// Delay-table builder (host, IEEE float64, compiled without FP contraction).
//
// Per iteration l = 1..log2(Nf) and sub-band j, the merged band [f0, f2) is
// split at its border frequency f1 (Sec. 4, addition rule; the border reading
// is the one Sec. 4.2 gives for unequal sub-bands). Its row dt reads
//   the lower half [f0, f1) at row d_lo = t0 - t1 = round(dt * C_{f2,f0}) and
//   the upper half [f1, f2) at row d_hi = t1 - t2 = dt - d_lo, shifted by d_lo,
// with C_{f2,f0} from Eq. (Cf2f0). Rows are counted top-down from the Nd
// output rows: a child needs exactly the rows its parent reads, which is the
// discrete counterpart of the dt_max(i, f0) estimate of Algorithm 1.
//
// Other delay laws dt ~ f^gamma (Sec. 4.2, other functional forms) change
// only C: the power -2 of Eq. (Cf2f0) becomes gamma.
//
// Nf need not be a power of two (Sec. 4.2, the case Nf != 2^k): the tree
// keeps 2^ceil(log2 Nf) channel positions, and the positions past the last
// channel are zero-width bands at its upper edge with no data. A merge whose
// upper half is such a band has C = 1 exactly, so its rows are the lower
// half's rows plus a zero: the lower half passes through unchanged. Every
// other merge splits a band of unequal halves at their border, f2 being the
// upper edge of its last channel. Bands without a channel have one row.
//
// The two-C rule (Sec. 4.2, rounding and binning; `rule` 1) treats a
// channel as the point of its label (lower edge) e_k, a sub-band's delay
// running from its first channel's label to its last's. A merge of channels
// k0..km-1 and km..k1 then computes C twice over the label span [e_k0, e_k1]:
// with the lower sub-band's end frequency e_{km-1} for the lower half's delay
// d_lo, and with the upper sub-band's start frequency e_km for the upper
// half's shift s (its delay being dt - s), so the curve's travel between the
// two labels is the gap s - d_lo. A single channel spans no delay: every
// channel needs only row 0.
//
// A known smallest delay d_min (Sec. 4.2, different range of dispersions) is
// a frequency-dependent shift of the input: channel k is delayed by
// pre_k = round(d_min * phi(c_k)) samples, phi(f) = (f_min^g - f^g) /
// (f_min^g - f_max^g) the fraction of the band delay reached at its centre
// c_k, after which output row dt follows total delay d_min + dt (the run a
// row adds in channel k is then centred on the curve's passage through it).
#include "fdmt_tables.h"

#include <algorithm>
#include <cmath>

namespace fdmt {

namespace {

// f^gamma; the cold-plasma law's f^-2 as 1 / (f * f).
double law(double f, double gamma) { return gamma == -2.0 ? 1.0 / (f * f) : std::pow(f, gamma); }

// Eq. (Cf2f0), evaluated exactly in this order.
double merge_coefficient(double f0, double f1, double f2, double gamma) {
  const double num = law(f1, gamma) - law(f0, gamma);
  const double den = law(f2, gamma) - law(f0, gamma);
  return num / den;
}

// Nearest integer, ties upward; x >= 0 here.
int32_t round_half_up(double x) { return static_cast<int32_t>(std::floor(x + 0.5)); }

} // namespace

std::string build_tables(Tables &t, int nf, int nd, double f_min, double f_max, double gamma, int d_min,
                         int rule) {
  if (nf < 1) return "Nf must be >= 1";
  if (nd < 1) return "Nd must be >= 1";
  if (!(f_min > 0.0) || !(f_max > f_min) || !std::isfinite(f_max))
    return "need 0 < f_min < f_max (finite)";
  if (!std::isfinite(gamma) || gamma == 0.0) return "the delay law's power must be finite and nonzero";
  if (d_min < 0) return "d_min must be >= 0";
  if (rule != 0 && rule != 1) return "rule must be 0 (one C) or 1 (two C's)";
  int levels = 0;
  while ((1 << levels) < nf) ++levels;
  const int slots = 1 << levels;

  t = Tables();
  t.nf = nf;
  t.nd = nd;
  t.levels = levels;
  t.slots = slots;
  t.f_min = f_min;
  t.f_max = f_max;
  t.gamma = gamma;
  t.d_min = d_min;
  t.rule = rule;

  const double df = (f_max - f_min) / nf;
  std::vector<double> edge(slots + 1);
  for (int k = 0; k <= slots; ++k) edge[k] = f_min + static_cast<double>(k <= nf ? k : nf) * df;

  t.rows.assign(levels + 1, {});
  t.d_lo.assign(levels + 1, {});
  t.d_hi.assign(levels + 1, {});
  t.shift.assign(levels + 1, {});
  t.rows[levels] = {nd};

  // Top-down: split every sub-band of iteration l, which fixes the row counts
  // of iteration l - 1.
  std::vector<std::vector<std::vector<int32_t>>> lo_of(levels + 1), hi_of(levels + 1), s_of(levels + 1);
  for (int l = levels; l >= 1; --l) {
    const int nsub = slots >> l;
    t.rows[l - 1].assign(2 * nsub, 0);
    lo_of[l].resize(nsub);
    hi_of[l].resize(nsub);
    s_of[l].resize(nsub);
    for (int j = 0; j < nsub; ++j) {
      const int64_t first = static_cast<int64_t>(j) << l, mid = static_cast<int64_t>(2 * j + 1) << (l - 1);
      const int64_t end = std::min<int64_t>(static_cast<int64_t>(j + 1) << l, nf);  // past its last channel
      double c_lo, c_hi;
      if (first >= nf) {
        c_lo = c_hi = 0.0;  // a band with no channel has only row 0, which any C maps to 0
      } else if (mid >= nf) {
        c_lo = c_hi = 1.0;  // no channel in the upper half: the band is its lower half
      } else if (rule == 0) {
        c_lo = c_hi = merge_coefficient(edge[first], edge[mid], edge[end], gamma);
      } else {
        c_lo = merge_coefficient(edge[first], edge[mid - 1], edge[end - 1], gamma);
        c_hi = merge_coefficient(edge[first], edge[mid], edge[end - 1], gamma);
      }
      const int32_t n = t.rows[l][j];
      auto &lo = lo_of[l][j];
      auto &hi = hi_of[l][j];
      auto &sh = s_of[l][j];
      lo.resize(n);
      hi.resize(n);
      sh.resize(n);
      for (int32_t dt = 0; dt < n; ++dt) {
        const int32_t d = round_half_up(static_cast<double>(dt) * c_lo);
        const int32_t sv = round_half_up(static_cast<double>(dt) * c_hi);
        if (d < 0 || d > dt || sv < 0 || sv > dt) return "merge coefficient outside [0, 1]";
        lo[dt] = d;
        sh[dt] = sv;
        hi[dt] = dt - sv;
      }
      t.rows[l - 1][2 * j] = lo[n - 1] + 1;
      t.rows[l - 1][2 * j + 1] = hi[n - 1] + 1;
    }
  }

  // Row offsets of every plane.
  t.row_off.assign(levels + 1, {});
  t.total.assign(levels + 1, 0);
  for (int l = 0; l <= levels; ++l) {
    int64_t acc = 0;
    t.row_off[l].resize(t.rows[l].size());
    for (size_t j = 0; j < t.rows[l].size(); ++j) {
      t.row_off[l][j] = acc;
      acc += t.rows[l][j];
    }
    t.total[l] = acc;
    if (acc > INT32_MAX) return "plane too tall";
  }

  // Flat per-row tables.
  t.merge.assign(levels + 1, {});
  t.adj.assign(levels + 1, {});
  for (int l = 1; l <= levels; ++l) {
    const int nsub = slots >> l;
    auto &m = t.merge[l];
    m.resize(t.total[l]);
    t.d_lo[l].resize(t.total[l]);
    t.d_hi[l].resize(t.total[l]);
    t.shift[l].resize(t.total[l]);
    auto &a = t.adj[l];
    a.assign(t.total[l - 1], AdjRow{0, 0, 0, 0});
    for (int j = 0; j < nsub; ++j) {
      const int64_t base = t.row_off[l][j];
      const int64_t lo_base = t.row_off[l - 1][2 * j];
      const int64_t hi_base = t.row_off[l - 1][2 * j + 1];
      for (int32_t dt = 0; dt < t.rows[l][j]; ++dt) {
        const int32_t dl = lo_of[l][j][dt], dh = hi_of[l][j][dt], sv = s_of[l][j][dt];
        const int64_t r = base + dt;
        m[r] = MergeRow{static_cast<int32_t>(lo_base + dl), static_cast<int32_t>(hi_base + dh), sv, j};
        t.d_lo[l][r] = dl;
        t.d_hi[l][r] = dh;
        t.shift[l][r] = sv;
        // Inverse maps: the parents of a child row are consecutive because
        // both d_lo and d_hi are non-decreasing in dt.
        AdjRow &al = a[lo_base + dl];
        if (al.count == 0) { al.first = static_cast<int32_t>(r); al.upper = 0; }
        if (al.first + al.count != r) return "lower-half inverse map not contiguous";
        ++al.count;
        AdjRow &ah = a[hi_base + dh];
        if (ah.count == 0) { ah.first = static_cast<int32_t>(r); ah.upper = 1; }
        if (ah.first + ah.count != r) return "upper-half inverse map not contiguous";
        ++ah.count;
      }
    }
    for (const AdjRow &x : a)
      if (x.count == 0) return "child row with no parent";
  }

  t.leaf_off.resize(slots);
  t.leaf_rows.resize(slots);
  for (int k = 0; k < slots; ++k) {
    t.leaf_off[k] = static_cast<int32_t>(t.row_off[0][k]);
    t.leaf_rows[k] = t.rows[0][k];
  }
  t.pre.assign(slots, kNoChannelPre);
  for (int k = 0; k < nf; ++k) t.pre[k] = 0;
  if (d_min > 0) {
    const double den = law(f_min, gamma) - law(f_max, gamma);
    for (int k = 0; k < nf; ++k) {
      const double centre = 0.5 * (edge[k] + edge[k + 1]);
      const double phi = (law(f_min, gamma) - law(centre, gamma)) / den;
      t.pre[k] = round_half_up(static_cast<double>(d_min) * phi);
      if (t.pre[k] < 0 || t.pre[k] > d_min) return "pre-shift outside [0, d_min]";
    }
  }
  return "";
}

} // namespace fdmt
