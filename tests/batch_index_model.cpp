// CPU model of the index arithmetic of the batched traversal (csrc/msbfs.hip:
// k_ms_seed, the level fills, td_phase, bu_phase with their hub pieces,
// hub_of, commit_atomic, step_parents) and of the hub list Kernel 1 builds for
// it, run sequentially with every array access bounds-checked.  Wavefront
// operations (ballots, shuffles, the hub pieces spread over wavefronts) are
// replayed lane by lane in the order a wavefront would see them.
//
// Input (binary, little endian): int64 n, int64 nnz, int64 row_ptr[n + 1],
// int32 col_idx[nnz]; then int32 k, int64 roots[k].  Arguments: input file,
// direction (0 auto, 1 top-down, 2 bottom-up), alpha, parents (0/1),
// waves (the number of wavefronts of the modelled grid), output file.
// Output: int8 levels[k][n].  Exit status 3 on an access out of bounds.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

namespace {

constexpr int kWave = 64;
constexpr int kLaneRow = 32;
constexpr int kRowBatch = 8;
constexpr int64_t kHubDeg = 4096;
constexpr int64_t kHubChunk = 1024;

template <class T>
struct Checked {
  const char *name;
  std::vector<T> v;
  Checked(const char *nm, size_t len, T init) : name(nm), v(len, init) {}
  T &operator[](int64_t i) {
    if (i < 0 || i >= (int64_t)v.size()) {
      std::fprintf(stderr, "out of bounds: %s[%lld] (size %zu)\n", name, (long long)i, v.size());
      std::exit(3);
    }
    return v[(size_t)i];
  }
};

int ffs64(uint64_t x) { return __builtin_ffsll((long long)x); }

struct Model {
  int64_t n, nnz;
  int k;
  bool par;
  int dir;
  double alpha;
  int64_t waves;
  uint64_t full;
  Checked<int64_t> rp;
  Checked<int32_t> ci;
  Checked<uint64_t> seen, buf0, buf1, buf2;
  Checked<int8_t> levels;
  Checked<int32_t> parents;
  Checked<int32_t> hint;
  Checked<int32_t> hub_list;
  Checked<uint64_t> hub_off;
  int64_t num_hubs = 0, hub_chunks = 0;
  uint64_t nf = 0, mf = 0, dec = 0;  // the next level's counters

  Model(int64_t n_, int64_t nnz_, int k_)
      : n(n_), nnz(nnz_), k(k_), rp("row_ptr", n_ + 1, 0), ci("col_idx", nnz_, 0),
        seen("seen", n_, 0), buf0("buf0", n_, 0), buf1("buf1", n_, 0), buf2("buf2", n_, 0),
        levels("levels", (size_t)k_ * n_, 0), parents("parents", (size_t)k_ * n_, 0),
        hint("hint", n_, -1), hub_list("hub_list", 0, 0), hub_off("hub_off", 1, 0) {
    full = k == 64 ? ~0ull : ((1ull << k) - 1);
  }

  // Kernel 1's hub list and piece offsets, and the hint (highest degree, then
  // smaller id, over the whole row)
  void aux() {
    std::vector<int32_t> hubs;
    for (int64_t v = 0; v < n; ++v)
      if (rp[v + 1] - rp[v] > kHubDeg) hubs.push_back((int32_t)v);
    num_hubs = (int64_t)hubs.size();
    hub_list = Checked<int32_t>("hub_list", hubs.size() ? hubs.size() : 1, 0);
    for (size_t i = 0; i < hubs.size(); ++i) hub_list[(int64_t)i] = hubs[i];
    hub_off = Checked<uint64_t>("hub_off", hubs.size() + 1, 0);
    for (int64_t i = 0; i < num_hubs; ++i) {
      const int32_t v = hub_list[i];
      hub_off[i + 1] = hub_off[i] + (uint64_t)((rp[v + 1] - rp[v] + kHubChunk - 1) / kHubChunk);
    }
    hub_chunks = (int64_t)hub_off[num_hubs];
    for (int64_t v = 0; v < n; ++v) {
      uint64_t best = 0;
      for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
        const int32_t u = ci[e];
        const uint64_t key =
            ((uint64_t)(rp[u + 1] - rp[u]) << 32) | (uint64_t)(0x7fffffffu - (uint32_t)u);
        if (key > best) best = key;
      }
      hint[v] = best ? (int32_t)(0x7fffffffu - (uint32_t)(best & 0xffffffffu)) : -1;
    }
  }

  int64_t hub_of(uint64_t c) {
    int64_t lo = 0, hi = num_hubs;
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (hub_off[mid] <= c) lo = mid; else hi = mid;
    }
    return lo;
  }

  void commit(int64_t v, uint64_t won, uint64_t old, int32_t p, int8_t lvl, bool with_par) {
    const uint64_t ps = seen[v];
    seen[v] = ps | won;
    int64_t d = -1;
    if (old == 0) {
      d = rp[v + 1] - rp[v];
      nf += 1;
      mf += (uint64_t)d;
    }
    if ((ps | won) == full && ps != full) {
      if (d < 0) d = rp[v + 1] - rp[v];
      dec += (uint64_t)d;
    }
    while (won) {
      const int b = ffs64(won) - 1;
      won &= won - 1;
      levels[(int64_t)b * n + v] = lvl;
      if (with_par) parents[(int64_t)b * n + v] = p;
    }
  }

  void td_edge(Checked<uint64_t> &next, int32_t u, uint64_t fu, int32_t v, int8_t lvl) {
    const uint64_t nw = fu & ~seen[v];
    if (!nw) return;
    const uint64_t old = next[v];
    next[v] = old | nw;
    const uint64_t won = nw & ~old;
    if (won) commit(v, won, old, u, lvl, par);
  }

  void td_phase(Checked<uint64_t> &front, Checked<uint64_t> &next, int8_t lvl) {
    const int64_t W = (n + kWave - 1) / kWave;
    for (int64_t gw = 0; gw < waves; ++gw)
      for (int64_t w = gw; w < W; w += waves) {
        uint64_t f[kWave];
        int64_t b[kWave], e[kWave];
        bool any = false;
        for (int l = 0; l < kWave; ++l) {
          const int64_t u = w * kWave + l;
          f[l] = u < n ? front[u] : 0;
          any |= f[l] != 0;
          b[l] = e[l] = 0;
          if (f[l]) {
            b[l] = rp[u];
            e[l] = rp[u + 1];
          }
        }
        if (!any) continue;
        for (int l = 0; l < kWave; ++l) {
          const int64_t d = e[l] - b[l];
          if (!(f[l] && d <= kLaneRow)) continue;
          const int32_t u = (int32_t)(w * kWave + l);
          for (int64_t k0 = b[l]; k0 < e[l]; k0 += kRowBatch) {
            int32_t vv[kRowBatch];
            uint64_t nw[kRowBatch], old[kRowBatch];
            for (int t = 0; t < kRowBatch; ++t) vv[t] = k0 + t < e[l] ? ci[k0 + t] : -1;
            for (int t = 0; t < kRowBatch; ++t) nw[t] = vv[t] >= 0 ? f[l] & ~seen[vv[t]] : 0ull;
            for (int t = 0; t < kRowBatch; ++t) {
              old[t] = ~0ull;
              if (nw[t]) {
                old[t] = next[vv[t]];
                next[vv[t]] = old[t] | nw[t];
              }
            }
            for (int t = 0; t < kRowBatch; ++t) {
              const uint64_t won = nw[t] & ~old[t];
              if (won) commit(vv[t], won, old[t], u, lvl, par);
            }
          }
        }
        for (int L = 0; L < kWave; ++L) {
          const int64_t d = e[L] - b[L];
          if (!(f[L] && d > kLaneRow && d <= kHubDeg)) continue;
          const int32_t uL = (int32_t)(w * kWave + L);
          for (int64_t c = b[L]; c < e[L]; c += kWave)
            for (int l = 0; l < kWave && c + l < e[L]; ++l) td_edge(next, uL, f[L], ci[c + l], lvl);
        }
      }
    for (int64_t gw = 0; gw < waves; ++gw)
      for (int64_t c = gw; c < hub_chunks; c += waves) {
        const int64_t i = hub_of((uint64_t)c);
        const int32_t h = hub_list[i];
        const uint64_t fh = front[h];
        if (!fh) continue;
        const int64_t kb = rp[h] + (int64_t)((uint64_t)c - hub_off[i]) * kHubChunk;
        const int64_t ke = std::min<int64_t>(kb + kHubChunk, rp[h + 1]);
        for (int64_t kk = kb; kk < ke; ++kk) td_edge(next, h, fh, ci[kk], lvl);
      }
  }

  // step_parents: per bit, the lowest lane of the step providing it
  void step_parents(int64_t v, uint64_t found, const uint64_t *g, const int32_t *u) {
    if (!par) return;
    while (found) {
      const int b = ffs64(found) - 1;
      found &= found - 1;
      for (int l = 0; l < kWave; ++l)
        if ((g[l] >> b) & 1) {
          parents[(int64_t)b * n + v] = u[l];
          break;
        }
    }
  }

  void bu_phase(Checked<uint64_t> &front, Checked<uint64_t> &next, int8_t lvl) {
    const int64_t W = (n + kWave - 1) / kWave;
    for (int64_t gw = 0; gw < waves; ++gw)
      for (int64_t w = gw; w < W; w += waves) {
        uint64_t s[kWave], got[kWave], missing[kWave];
        int64_t b[kWave], e[kWave];
        bool act[kWave], any = false;
        for (int l = 0; l < kWave; ++l) {
          const int64_t v = w * kWave + l;
          s[l] = v < n ? seen[v] : full;
          b[l] = e[l] = 0;
          if (s[l] != full) {
            b[l] = rp[v];
            e[l] = rp[v + 1];
          }
          const int64_t d = e[l] - b[l];
          act[l] = s[l] != full && d > 0 && d <= kHubDeg;
          any |= act[l];
          missing[l] = full & ~s[l];
          got[l] = 0;
        }
        if (!any) continue;
        for (int l = 0; l < kWave; ++l) {
          const int64_t v = w * kWave + l;
          const int64_t d = e[l] - b[l];
          if (act[l]) {
            const int32_t h = hint[v];
            if (h >= 0) {
              got[l] = front[h] & missing[l];
              uint64_t x = got[l];
              while (par && x) {
                const int bb = ffs64(x) - 1;
                x &= x - 1;
                parents[(int64_t)bb * n + v] = h;
              }
            }
          }
          if (act[l] && d <= kLaneRow && got[l] != missing[l]) {
            for (int64_t k0 = b[l]; k0 < e[l] && got[l] != missing[l]; k0 += kRowBatch) {
              int32_t uu[kRowBatch];
              uint64_t fu[kRowBatch];
              for (int t = 0; t < kRowBatch; ++t) uu[t] = k0 + t < e[l] ? ci[k0 + t] : -1;
              for (int t = 0; t < kRowBatch; ++t) fu[t] = uu[t] >= 0 ? front[uu[t]] : 0ull;
              for (int t = 0; t < kRowBatch; ++t) {
                const uint64_t g = fu[t] & missing[l] & ~got[l];
                if (g) {
                  got[l] |= g;
                  uint64_t x = g;
                  while (par && x) {
                    const int bb = ffs64(x) - 1;
                    x &= x - 1;
                    parents[(int64_t)bb * n + v] = uu[t];
                  }
                }
              }
            }
          }
        }
        for (int L = 0; L < kWave; ++L) {
          const int64_t d = e[L] - b[L];
          if (!(act[L] && d > kLaneRow && got[L] != missing[L])) continue;
          const int64_t vL = w * kWave + L;
          uint64_t gotL = got[L];
          for (int64_t c = b[L]; c < e[L]; c += kWave) {
            int32_t u[kWave];
            uint64_t g[kWave], orr = 0;
            for (int l = 0; l < kWave; ++l) {
              const int64_t kk = c + l;
              u[l] = -1;
              g[l] = 0;
              if (kk < e[L]) {
                u[l] = ci[kk];
                g[l] = front[u[l]] & missing[L];
              }
              orr |= g[l];
            }
            const uint64_t fresh = orr & ~gotL;
            if (fresh) {
              step_parents(vL, fresh, g, u);
              gotL |= fresh;
              if (gotL == missing[L]) break;
            }
          }
          got[L] = gotL;
        }
        for (int l = 0; l < kWave; ++l) {
          const int64_t v = w * kWave + l;
          if (got[l]) {
            next[v] = got[l];
            seen[v] = s[l] | got[l];
            const int64_t d = e[l] - b[l];
            nf += 1;
            mf += (uint64_t)d;
            if ((s[l] | got[l]) == full) dec += (uint64_t)d;
          }
        }
        for (int l = 0; l < kWave; ++l) {
          const int64_t v = w * kWave + l;
          uint64_t x = got[l];
          while (x) {
            const int bb = ffs64(x) - 1;
            x &= x - 1;
            levels[(int64_t)bb * n + v] = lvl;
          }
        }
      }
    for (int64_t gw = 0; gw < waves; ++gw)
      for (int64_t c = gw; c < hub_chunks; c += waves) {
        const int64_t i = hub_of((uint64_t)c);
        const int32_t h = hub_list[i];
        const uint64_t sh = seen[h];
        if (sh == full) continue;
        const uint64_t mh = full & ~sh;
        const int64_t kb = rp[h] + (int64_t)((uint64_t)c - hub_off[i]) * kHubChunk;
        const int64_t ke = std::min<int64_t>(kb + kHubChunk, rp[h + 1]);
        uint64_t gotc = 0;
        for (int64_t cc = kb; cc < ke; cc += kWave) {
          int32_t u[kWave];
          uint64_t g[kWave], orr = 0;
          for (int l = 0; l < kWave; ++l) {
            const int64_t kk = cc + l;
            u[l] = -1;
            g[l] = 0;
            if (kk < ke) {
              u[l] = ci[kk];
              g[l] = front[u[l]] & mh;
            }
            orr |= g[l];
          }
          const uint64_t fresh = orr & ~gotc;
          if (!fresh) continue;
          gotc |= fresh;
          const uint64_t old = next[h];
          next[h] = old | fresh;
          const uint64_t won = fresh & ~old;
          if (won) {
            step_parents(h, won, g, u);
            commit(h, won, old, -1, lvl, false);
          }
          if (gotc == mh) break;
        }
      }
  }
};

}  // namespace

int main(int argc, char **argv) {
  if (argc < 7) {
    std::fprintf(stderr, "usage: in dir alpha parents waves out\n");
    return 2;
  }
  FILE *f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t n = 0, nnz = 0;
  if (std::fread(&n, 8, 1, f) != 1 || std::fread(&nnz, 8, 1, f) != 1) return 2;
  std::vector<int64_t> rp(n + 1);
  std::vector<int32_t> ci(nnz);
  if (std::fread(rp.data(), 8, n + 1, f) != (size_t)(n + 1)) return 2;
  if (nnz && std::fread(ci.data(), 4, nnz, f) != (size_t)nnz) return 2;
  int32_t k = 0;
  if (std::fread(&k, 4, 1, f) != 1 || k < 1 || k > 64) return 2;
  std::vector<int64_t> roots(k);
  if (std::fread(roots.data(), 8, k, f) != (size_t)k) return 2;
  std::fclose(f);

  Model m(n, nnz, k);
  m.dir = std::atoi(argv[2]);
  m.alpha = std::atof(argv[3]);
  m.par = std::atoi(argv[4]) != 0;
  m.waves = std::atoll(argv[5]);
  for (int64_t i = 0; i <= n; ++i) m.rp[i] = rp[(size_t)i];
  for (int64_t i = 0; i < nnz; ++i) m.ci[i] = ci[(size_t)i];
  m.aux();
  // the fills: levels and parents -1, masks zero
  for (int64_t i = 0; i < (int64_t)k * n; ++i) {
    m.levels[i] = -1;
    m.parents[i] = -1;
  }
  // k_ms_seed
  uint64_t nf = 0, mf = 0;
  for (int b = 0; b < k; ++b) {
    const int64_t v = roots[(size_t)b];
    m.seen[v] |= 1ull << b;
    m.buf0[v] |= 1ull << b;
    m.levels[(int64_t)b * n + v] = 0;
    if (m.par) m.parents[(int64_t)b * n + v] = (int32_t)v;
    bool first = true;
    for (int c = 0; c < b; ++c)
      if (roots[(size_t)c] == v) first = false;
    if (first) {
      nf += 1;
      mf += (uint64_t)(m.rp[v + 1] - m.rp[v]);
    }
  }
  bool all = true;
  for (int c = 1; c < k; ++c) all &= roots[(size_t)c] == roots[0];
  uint64_t mu = (uint64_t)(m.rp[n] - (all ? m.rp[roots[0] + 1] - m.rp[roots[0]] : 0));
  Checked<uint64_t> *bufs[3] = {&m.buf0, &m.buf1, &m.buf2};
  int status = 0;
  for (int l = 0; nf != 0; ++l) {
    if (l > 126) {  // deeper than int8 levels hold
      status = 4;
      break;
    }
    const bool td = m.dir == 1 || (m.dir == 0 && (double)mf <= (double)mu / m.alpha);
    Checked<uint64_t> &front = *bufs[l % 3], &next = *bufs[(l + 1) % 3], &clr = *bufs[(l + 2) % 3];
    for (int64_t v = 0; v < n; ++v) clr[v] = 0;
    m.nf = m.mf = m.dec = 0;
    if (td)
      m.td_phase(front, next, (int8_t)(l + 1));
    else
      m.bu_phase(front, next, (int8_t)(l + 1));
    nf = m.nf;
    mf = m.mf;
    mu -= m.dec;
  }
  FILE *o = std::fopen(argv[6], "wb");
  if (!o) return 2;
  std::fwrite(m.levels.v.data(), 1, m.levels.v.size(), o);
  if (m.par) std::fwrite(m.parents.v.data(), 4, m.parents.v.size(), o);
  std::fclose(o);
  return status;
}
