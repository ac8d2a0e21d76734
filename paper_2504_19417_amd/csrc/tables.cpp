// Host-side set-up of the encoder: parameter checks, the half-window offset
// list, the FP64-built offset-phase table and its matrix-core layout.
//
// The phase of a neighbour at integer offset o = (dx, dy, dt) from the query
// is theta_j(o) = A[j] . o (Eqn. 10 with A holding the per-axis frequencies
// already divided by the radii, Algorithm 1 frequency draw).  Algorithm 1
// precomputes the spatial factor because offsets are integers with a finite
// range; the same holds for dt once time is binned, so the whole factor
// e^{i theta_j(o)} is tabulated once per context.  Since e^{-i theta} is the
// conjugate of e^{i theta}, the window sum over o and -o only needs
// cos(theta) on the pair sum of counts and sin(theta) on their difference,
// which halves the table (and the contraction) to the centre plus the
// lexicographically positive half of the window.
#include <cmath>
#include <cstring>
#include <limits>

#include "veckm_internal.h"

namespace veckm {

static bool valid_d(int d) {
  return d == 16 || d == 32 || d == 48 || d == 64 || d == 128 || d == 256;
}

int check_params(const veckm_params* p) {
  if (!p || !p->A) return VECKM_E_INVAL;
  if (p->width < 1 || p->height < 1 || p->max_bins < 1) return VECKM_E_INVAL;
  if (p->rx < 0 || p->rx > kMaxRxy || p->ry < 0 || p->ry > kMaxRxy) return VECKM_E_INVAL;
  if (p->rt < -1 || p->rt > kMaxRt) return VECKM_E_INVAL;
  if (p->rt == -1 && p->max_bins > kMaxPaperBins) return VECKM_E_INVAL;
  if (!valid_d(p->d)) return VECKM_E_INVAL;
  if (p->precision != VECKM_FP32 && p->precision != VECKM_FP16) return VECKM_E_INVAL;
  if (p->max_events < 1 || p->max_events > (int64_t)std::numeric_limits<int32_t>::max())
    return VECKM_E_INVAL;
  const int64_t V = (int64_t)p->width * p->height * p->max_bins;
  if (V > (int64_t)std::numeric_limits<int32_t>::max() / 2) return VECKM_E_INVAL;
  for (int i = 0; i < 3 * p->d; ++i)
    if (!std::isfinite(p->A[i])) return VECKM_E_INVAL;
  if (p->rt >= 0) {
    // the encoder needs a brick whose count box fits in LDS beside two
    // table slabs (large D with the largest windows does not)
    const SlotTable st = make_slots(p->rx, p->ry, p->rt);
    Brick b;
    int nbuf;
    if (!choose_layout(p->rx, p->ry, p->rt, p->d, p->precision, st.KP, &b, &nbuf))
      return VECKM_E_INVAL;
  }
  return VECKM_OK;
}

OffsetTable make_offsets(int rx, int ry, int rt) {
  OffsetTable t;
  t.off = {0, 0, 0};  // centre
  for (int dt = 0; dt <= rt; ++dt)
    for (int dy = (dt == 0 ? 0 : -ry); dy <= ry; ++dy)
      for (int dx = (dt == 0 && dy == 0 ? 1 : -rx); dx <= rx; ++dx) {
        t.off.push_back(dx);
        t.off.push_back(dy);
        t.off.push_back(dt);
      }
  t.K = (int)t.off.size() / 3;
  t.KP = (t.K + kKStep - 1) / kKStep * kKStep;
  return t;
}

uint16_t fp16_bits_rne(double v) {
  if (std::isnan(v)) return 0x7e00;
  const uint16_t sign = std::signbit(v) ? 0x8000 : 0;
  const double a = std::fabs(v);
  if (a == 0.0) return sign;
  if (a >= 65520.0) return sign | 0x7c00;  // rounds to infinity
  int e;
  std::frexp(a, &e);  // a = f * 2^e, f in [0.5, 1)
  if (e - 1 >= -14) {  // normal: 1.m * 2^(e-1)
    double r = std::nearbyint(std::ldexp(a, 10 - (e - 1)));  // in [1024, 2048]
    int E = e - 1 + 15;
    if (r >= 2048.0) { r *= 0.5; E += 1; }
    if (E >= 31) return sign | 0x7c00;
    return (uint16_t)(sign | (E << 10) | ((int)r - 1024));
  }
  // subnormal: multiples of 2^-24 (rounding up to 1024 gives the smallest normal)
  return (uint16_t)(sign | (int)std::nearbyint(std::ldexp(a, 24)));
}

double fp16_to_double(uint16_t h) {
  const int s = h >> 15, E = (h >> 10) & 31, M = h & 1023;
  double v;
  if (E == 0) v = std::ldexp((double)M, -24);
  else if (E == 31) v = M ? std::numeric_limits<double>::quiet_NaN()
                          : std::numeric_limits<double>::infinity();
  else v = std::ldexp((double)(M + 1024), E - 25);
  return s ? -v : v;
}

uint16_t bf16_bits_rne(float v) {
  uint32_t u;
  std::memcpy(&u, &v, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// cos/sin of the offset phase for table entry k and frequency j, in FP64.
static void phase(const OffsetTable& t, const double* A, int k, int j, double* c, double* s) {
  if (k == 0) {  // centre: met as +o and -o, so half of cos(0); sin(0) = 0
    *c = 0.5;
    *s = 0.0;
    return;
  }
  const double th = A[3 * j + 0] * (double)t.off[3 * k + 0] +
                    A[3 * j + 1] * (double)t.off[3 * k + 1] +
                    A[3 * j + 2] * (double)t.off[3 * k + 2];
  *c = std::cos(th);
  *s = std::sin(th);
}

void make_phase_bits(const OffsetTable& t, const double* A, int d, uint16_t* out) {
  for (int k = 0; k < t.K; ++k)
    for (int j = 0; j < d; ++j) {
      double c, s;
      phase(t, A, k, j, &c, &s);
      const uint16_t ch = fp16_bits_rne(c), sh = fp16_bits_rne(s);
      uint16_t* o = out + ((size_t)k * d + j) * 4;
      o[0] = ch;
      o[1] = fp16_bits_rne(c - fp16_to_double(ch));
      o[2] = sh;
      o[3] = fp16_bits_rne(s - fp16_to_double(sh));
    }
}

void make_paper_tables(const double* A, int d, int width, int height, int max_bins,
                       std::vector<float>* ttab, std::vector<float>* xtab,
                       std::vector<float>* ytab) {
  auto fill = [&](std::vector<float>* out, int lo, int hi, int col) {
    out->assign((size_t)(hi - lo + 1) * d * 2, 0.f);
    for (int o = lo; o <= hi; ++o)
      for (int j = 0; j < d; ++j) {
        const double th = A[3 * j + col] * (double)o;
        (*out)[((size_t)(o - lo) * d + j) * 2 + 0] = (float)std::cos(th);
        (*out)[((size_t)(o - lo) * d + j) * 2 + 1] = (float)std::sin(th);
      }
  };
  fill(ttab, 0, max_bins - 1, 2);
  fill(xtab, 0, width - 1, 0);
  fill(ytab, 0, height - 1, 1);
}

int lds_volume_halves(const Brick& b, int rx, int ry, int rt) {
  return (b.bx + 2 * rx) * (b.by + 2 * ry) * (b.bt + 2 * rt);
}



SlotTable make_slots(int rx, int ry, int rt) {
  SlotTable t;
  auto row = [&](int dx0, int dx1, int dy, int dt, bool centre) {
    const int n = dx1 - dx0 + 1, padded = (n + 3) / 4 * 4;
    for (int i = 0; i < padded; ++i) {
      const int dx = dx0 + i;
      const int kind = i >= n ? 0 : (centre && dx == 0 ? 2 : 1);
      t.slot.insert(t.slot.end(), {dx, dy, dt, kind});
      if (kind) ++t.K;
    }
  };
  row(0, rx, 0, 0, true);  // centre row: the centre and dx > 0
  for (int dt = 0; dt <= rt; ++dt)
    for (int dy = (dt == 0 ? 1 : -ry); dy <= ry; ++dy) row(-rx, rx, dy, dt, false);
  int n = (int)t.slot.size() / 4;
  t.KP = (n + kKStep - 1) / kKStep * kKStep;
  for (; n < t.KP; ++n) t.slot.insert(t.slot.end(), {0, 0, 0, 0});
  return t;
}

std::vector<uint16_t> make_slot_fragments(const SlotTable& t, const double* A, int d, int na) {
  const int nt_total = d / 16, ksteps = t.KP / kKStep;
  std::vector<uint16_t> frag((size_t)ksteps * na * nt_total * 64 * 8, 0);
  size_t idx = 0;
  for (int ks = 0; ks < ksteps; ++ks)
    for (int a = 0; a < na; ++a)
      for (int nt = 0; nt < nt_total; ++nt)
        for (int lane = 0; lane < 64; ++lane)
          for (int e = 0; e < 8; ++e, ++idx) {
            const int k = ks * kKStep + 8 * (lane >> 4) + e;
            const int j = 16 * nt + (lane & 15);
            const int* s = &t.slot[4 * k];
            if (s[3] == 0) continue;
            double c = 0.5, sn = 0.0;  // centre: met as +o and -o
            if (s[3] == 1) {
              const double th = A[3 * j + 0] * (double)s[0] + A[3 * j + 1] * (double)s[1] +
                                A[3 * j + 2] * (double)s[2];
              c = std::cos(th);
              sn = std::sin(th);
            }
            const double v = (na == 4 ? (a < 2) : (a == 0)) ? c : sn;
            const uint16_t hi = fp16_bits_rne(v);
            const bool lo = na == 4 && (a & 1);
            frag[idx] = lo ? fp16_bits_rne(v - fp16_to_double(hi)) : hi;
          }
  return frag;
}

std::vector<int32_t> make_run_offsets(const SlotTable& t, const Brick& b, int rx, int ry) {
  const int SX = box_sx(b, rx), SY = b.by + 2 * ry;
  std::vector<int32_t> runs(t.KP / 4, 0);
  for (int r = 0; r < t.KP / 4; ++r) {
    const int* s = &t.slot[4 * 4 * r];
    runs[r] = (s[2] * SY + s[1]) * SX + s[0];
  }
  return runs;
}

std::vector<uint16_t> make_slot_weights(const SlotTable& t) {
  std::vector<uint16_t> w(t.KP, 0);
  for (int k = 0; k < t.KP; ++k) {
    const int kind = t.slot[4 * k + 3];
    w[k] = kind == 0 ? 0 : (kind == 2 ? fp16_bits_rne(0.5) : fp16_bits_rne(1.0));
  }
  return w;
}

// Brick and number of phase-table slabs buffered in LDS: the largest brick
// that fits beside two slabs, then as many slabs (up to four) as fit beside
// it.  Larger bricks amortise the window halo, fill the row chunks better and
// cut the number of passes over the table; extra slabs hide the latency of
// the table copies (three or four need the copies split evenly over the
// waves).
bool choose_layout(int rx, int ry, int rt, int d, int precision, int kp, Brick* brick,
                   int* nbuf) {
  const Brick cand[] = {{32, 16, 8}, {32, 16, 4}, {16, 16, 8}, {16, 16, 4},
                        {16, 8, 4},  {8, 8, 4},   {8, 8, 2},   {8, 4, 2}, {4, 4, 1}};
  const int na = precision == VECKM_FP32 ? 4 : 2;
  const bool even = (na * (d / 16) * 64) % (encode_waves() * 64) == 0;  // copies split evenly
  auto fits = [&](const Brick& b, int nb) {
    return box_sx(b, rx) <= 64 &&
           encode_lds_need(d, precision, nb, kp, box_dwords(b, rx, ry, rt)) <= 160 * 1024;
  };
  for (const Brick& b : cand)
    if (fits(b, 2)) {
      *brick = b;
      *nbuf = 2;
      for (int nb = even ? kMaxSlabBuffers : 2; nb > 2; --nb)
        if (fits(b, nb)) {
          *nbuf = nb;
          break;
        }
      return true;
    }
  *brick = Brick{4, 4, 1};
  *nbuf = 2;
  return false;
}

// The encoder tilings a context offers: the default layout above first,
// then each larger brick whose count box still fits beside two slabs (with
// as many slabs as fit), then a smaller brick if it fits more slabs than the
// default.  Larger bricks pay off where bricks hold few query voxels (sparse
// slices: fewer passes over the table per row); deeper slab buffering where
// they hold many.
std::vector<Tiling> tiling_candidates(int rx, int ry, int rt, int d, int precision, int kp) {
  std::vector<Tiling> out(1);
  choose_layout(rx, ry, rt, d, precision, kp, &out[0].brick, &out[0].nbuf);
  const Tiling def = out[0];
  const Brick cand[] = {{32, 32, 8}, {32, 16, 16}, {32, 16, 4}};
  const int na = precision == VECKM_FP32 ? 4 : 2;
  const bool even = (na * (d / 16) * 64) % (encode_waves() * 64) == 0;
  for (const Brick& b : cand) {
    const bool bigger = b.volume() > def.brick.volume();
    if (b.volume() == def.brick.volume() || b.volume() > kMaxBrickVoxels || box_sx(b, rx) > 64)
      continue;
    auto fits = [&](int nb) {
      return encode_lds_need(d, precision, nb, kp, box_dwords(b, rx, ry, rt)) <= 160 * 1024;
    };
    if (!fits(2)) continue;
    Tiling t{b, 2};
    for (int nb = even ? kMaxSlabBuffers : 2; nb > 2; --nb)
      if (fits(nb)) {
        t.nbuf = nb;
        break;
      }
    if (!bigger && t.nbuf <= def.nbuf) continue;  // smaller only for deeper buffering
    out.push_back(t);
  }
  // each of them also with the other wave layouts (four frequency tiles or
  // more per wave: D >= 64), where they fit: 8 waves of 4 row tiles over half
  // the frequencies (1); 4 (2), 8 (3) or, at D <= 128, 16 (4) waves over
  // every frequency of their rows, whose loads are pipelined within each
  // wave with one slab in flight (and whose encoder can run the perceptron
  // itself)
  const size_t n = out.size();
  for (int layout = 1; layout <= 4; ++layout)
    for (size_t i = 0; i < n && d >= 64 && (layout < 4 || d <= 128); ++i) {
      Tiling t = out[i];
      t.layout = layout;
      if (layout >= 2) {
        t.nbuf = 2;
        bool dup = false;
        for (size_t k = n; k < out.size(); ++k)
          dup = dup || (out[k].layout == layout && out[k].brick.bx == t.brick.bx &&
                        out[k].brick.by == t.brick.by && out[k].brick.bt == t.brick.bt);
        if (dup) continue;
      }
      const bool even_l = (na * (d / 16) * 64) % (encode_waves(layout) * 64) == 0;
      if (t.nbuf > 2 && !even_l) continue;
      if (encode_lds_need(d, precision, t.nbuf, kp, box_dwords(t.brick, rx, ry, rt), layout) >
          160 * 1024)
        continue;
      out.push_back(t);
    }
  // where the encoder can run the perceptron itself (D = 64 or 128), the
  // 16-wave pipelined layout on the default brick comes first: the fused
  // perceptron keeps rows out of HBM, and on the 1M-event slice it runs
  // the FP32 form as fast as the 8-wave layout (0.46 ms after warm-up) and
  // the FP16 form's larger bricks about 4 % faster (0.31 against 0.32 ms;
  // the tuner picks those bricks when slices are long enough for them).
  if (d == 64 || d == 128) {
    const int want = 4;
    long pick = -1;
    for (size_t k = 1; k < out.size() && pick < 0; ++k) {
      const Tiling& t = out[k];
      if (t.layout == want && t.brick.bx == def.brick.bx && t.brick.by == def.brick.by &&
          t.brick.bt == def.brick.bt)
        pick = (long)k;
    }
    if (pick > 0) {
      const Tiling t = out[(size_t)pick];
      out.erase(out.begin() + pick);
      out.insert(out.begin(), t);
    }
  }
  return out;
}

std::vector<uint16_t> make_w1_fragments(const float* W1, int hidden, int d, int na, int shift) {
  const int nt = d / 16, terms = na / 2, msteps = hidden / 32, k2 = 2 * d;
  std::vector<uint16_t> frag((size_t)msteps * na * nt * 64 * 8, 0);
  size_t idx = 0;
  for (int ms = 0; ms < msteps; ++ms)
    for (int q = 0; q < na; ++q)
      for (int kk = 0; kk < nt; ++kk)
        for (int lane = 0; lane < 64; ++lane)
          for (int e = 0; e < 8; ++e, ++idx) {
            const int t = q / 2, tile = q % 2;
            const int h = (2 * ms + tile) * 16 + (lane & 15);
            const int g = lane >> 4;
            // feature: tile 2kk' (e < 4) or 2kk' + 1 (e >= 4) of the real
            // (kk < nt / 2) or imaginary parts, lane group g, element e % 4
            const int kp = kk % (nt / 2);
            const int f = (kk < nt / 2 ? 0 : d) + 32 * kp + 16 * (e >> 2) + 4 * g + (e & 3);
            const float w = W1[(size_t)h * k2 + f];
            if (terms == 1) {
              frag[idx] = bf16_bits_rne(w);
            } else {
              const double v = std::ldexp((double)w, shift);
              const uint16_t hi = fp16_bits_rne(v);
              frag[idx] = t == 0 ? hi : fp16_bits_rne(v - fp16_to_double(hi));
            }
          }
  return frag;
}

}  // namespace veckm
