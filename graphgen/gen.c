/*
 * Seeded synthetic bipartite graph generator (input side only).
 *
 * This file produces edge lists; it holds none of the butterfly-counting
 * arithmetic and is shared, read-only, by the CPU oracle and the GPU path.
 *
 * Published methods used, each written here from its definition:
 *   - SplitMix64 (Steele, Lea, Flood 2014) to expand a 64-bit seed.
 *   - xoshiro256** (Blackman, Vigna 2018) as the stream generator.
 *   - Vose's alias method (Vose 1991) for sampling proportional to weights.
 *   - Fisher-Yates (Durstenfeld 1964) for shuffles and partial selections.
 *   - LSD radix sort on 16-bit digits for de-duplicating pair keys.
 *
 * Everything is single threaded so the output depends only on the seed.
 * Edges are written as int32 pairs (upper, lower), 0-based per layer.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t s[4]; } gg_rng;

static uint64_t splitmix64(uint64_t* x) {
  uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static void rng_seed(gg_rng* r, uint64_t seed) {
  uint64_t x = seed;
  for (int i = 0; i < 4; ++i) r->s[i] = splitmix64(&x);
}

static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static inline uint64_t rng_next(gg_rng* r) {
  uint64_t* s = r->s;
  const uint64_t result = rotl(s[1] * 5, 7) * 9;
  const uint64_t t = s[1] << 17;
  s[2] ^= s[0];
  s[3] ^= s[1];
  s[1] ^= s[2];
  s[0] ^= s[3];
  s[2] ^= t;
  s[3] = rotl(s[3], 45);
  return result;
}

/* uniform double in [0,1) with 53 random bits */
static inline double rng_double(gg_rng* r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }

/* uniform integer in [0,n) by rejection (Lemire's multiply-shift with exact rejection) */
static inline uint64_t rng_below(gg_rng* r, uint64_t n) {
  if (n <= 1) return 0;
  uint64_t lim = (0 - n) % n; /* 2^64 mod n */
  for (;;) {
    uint64_t x = rng_next(r);
    __uint128_t mprod = (__uint128_t)x * n;
    uint64_t lo = (uint64_t)mprod;
    if (lo >= lim) return (uint64_t)(mprod >> 64);
  }
}

/* ---------------------------------------------------------------- alias */
typedef struct {
  int64_t n;
  double* prob;
  int32_t* alias;
} gg_alias;

static int alias_build(gg_alias* a, const double* w, int64_t n) {
  a->n = n;
  a->prob = (double*)malloc(sizeof(double) * (size_t)n);
  a->alias = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* small = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* large = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  double* p = (double*)malloc(sizeof(double) * (size_t)n);
  if (!a->prob || !a->alias || !small || !large || !p) return -1;
  double sum = 0;
  for (int64_t i = 0; i < n; ++i) sum += w[i];
  int64_t ns = 0, nl = 0;
  for (int64_t i = 0; i < n; ++i) {
    p[i] = w[i] * (double)n / sum;
    if (p[i] < 1.0) small[ns++] = (int32_t)i; else large[nl++] = (int32_t)i;
  }
  while (ns > 0 && nl > 0) {
    int32_t s = small[--ns];
    int32_t g = large[--nl];
    a->prob[s] = p[s];
    a->alias[s] = g;
    p[g] = (p[g] + p[s]) - 1.0;
    if (p[g] < 1.0) small[ns++] = g; else large[nl++] = g;
  }
  while (nl > 0) { int32_t g = large[--nl]; a->prob[g] = 1.0; a->alias[g] = g; }
  while (ns > 0) { int32_t s = small[--ns]; a->prob[s] = 1.0; a->alias[s] = s; }
  free(small); free(large); free(p);
  return 0;
}

static void alias_free(gg_alias* a) { free(a->prob); free(a->alias); }

static inline int64_t alias_draw(const gg_alias* a, gg_rng* r) {
  int64_t i = (int64_t)rng_below(r, (uint64_t)a->n);
  return rng_double(r) < a->prob[i] ? i : a->alias[i];
}

/* ------------------------------------------------------------- radix sort */
static int sort_u64(uint64_t* k, int64_t n, int bits) {
  if (n <= 1) return 0;
  uint64_t* tmp = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
  if (!tmp) return -1;
  int64_t* cnt = (int64_t*)malloc(sizeof(int64_t) * 65536);
  uint64_t* src = k;
  uint64_t* dst = tmp;
  for (int shift = 0; shift < bits; shift += 16) {
    memset(cnt, 0, sizeof(int64_t) * 65536);
    for (int64_t i = 0; i < n; ++i) cnt[(src[i] >> shift) & 0xFFFF]++;
    int64_t acc = 0;
    for (int d = 0; d < 65536; ++d) { int64_t c = cnt[d]; cnt[d] = acc; acc += c; }
    for (int64_t i = 0; i < n; ++i) dst[cnt[(src[i] >> shift) & 0xFFFF]++] = src[i];
    uint64_t* t = src; src = dst; dst = t;
  }
  if (src != k) memcpy(k, src, sizeof(uint64_t) * (size_t)n);
  free(tmp); free(cnt);
  return 0;
}

static int64_t unique_sorted(uint64_t* k, int64_t n) {
  if (n == 0) return 0;
  int64_t o = 1;
  for (int64_t i = 1; i < n; ++i) if (k[i] != k[o - 1]) k[o++] = k[i];
  return o;
}

static int bits_for(uint64_t x) { int b = 0; while (b < 64 && (x >> b)) ++b; return b < 1 ? 1 : b; }

/* ------------------------------------------------------ distinct pair set */
/*
 * Collects `need` distinct keys u*nL+v drawn iid from `draw` and absent from
 * the sorted `protect` list.  Surplus keys are dropped uniformly at random.
 * After `max_rounds` weighted rounds the remainder is drawn uniformly over
 * all cells, so the loop always ends when need <= cells - |protect|.
 */
typedef struct {
  const gg_alias* au;  /* NULL: uniform on the upper side */
  const gg_alias* al;  /* NULL: uniform on the lower side */
  int64_t nU, nL;
} gg_pairdist;

static inline uint64_t draw_key(const gg_pairdist* d, gg_rng* r, int uniform) {
  int64_t u = (!uniform && d->au) ? alias_draw(d->au, r) : (int64_t)rng_below(r, (uint64_t)d->nU);
  int64_t v = (!uniform && d->al) ? alias_draw(d->al, r) : (int64_t)rng_below(r, (uint64_t)d->nL);
  return (uint64_t)u * (uint64_t)d->nL + (uint64_t)v;
}

static int64_t collect_pairs(const gg_pairdist* d, gg_rng* r, int64_t need, const uint64_t* protect,
                             int64_t nprotect, uint64_t** out_set, int max_rounds) {
  int kbits = bits_for((uint64_t)d->nU * (uint64_t)d->nL);
  uint64_t* set = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(need > 0 ? need : 1));
  if (!set) return -1;
  int64_t have = 0;
  int round = 0;
  while (have < need) {
    int64_t want = need - have;
    int64_t k = want + want / 16 + 1024;
    uint64_t* cand = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)k);
    if (!cand) { free(set); return -1; }
    int uniform = round >= max_rounds;
    int64_t nc = 0;
    for (int64_t i = 0; i < k; ++i) cand[nc++] = draw_key(d, r, uniform);
    if (sort_u64(cand, nc, kbits)) { free(cand); free(set); return -1; }
    nc = unique_sorted(cand, nc);
    if (nprotect) { /* remove protected keys by a linear merge */
      int64_t p = 0, o = 0;
      for (int64_t i = 0; i < nc; ++i) {
        while (p < nprotect && protect[p] < cand[i]) ++p;
        if (p < nprotect && protect[p] == cand[i]) continue;
        cand[o++] = cand[i];
      }
      nc = o;
    }
    /* merge set (sorted, unique) with cand (sorted, unique), dropping repeats */
    uint64_t* merged = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(have + nc + 1));
    if (!merged) { free(cand); free(set); return -1; }
    int64_t i = 0, j = 0, o = 0;
    while (i < have && j < nc) {
      if (set[i] < cand[j]) merged[o++] = set[i++];
      else if (set[i] > cand[j]) merged[o++] = cand[j++];
      else { merged[o++] = set[i++]; ++j; }
    }
    while (i < have) merged[o++] = set[i++];
    while (j < nc) merged[o++] = cand[j++];
    free(cand); free(set);
    set = merged;
    have = o;
    ++round;
  }
  if (have > need) {
    /* drop (have - need) uniformly chosen elements */
    int64_t drop = have - need;
    uint8_t* mark = (uint8_t*)calloc((size_t)have, 1);
    if (!mark) { free(set); return -1; }
    for (int64_t t = 0; t < drop;) {
      int64_t idx = (int64_t)rng_below(r, (uint64_t)have);
      if (!mark[idx]) { mark[idx] = 1; ++t; }
    }
    int64_t o = 0;
    for (int64_t i = 0; i < have; ++i) if (!mark[i]) set[o++] = set[i];
    free(mark);
    have = o;
  }
  *out_set = set;
  return have;
}

static void shuffle_u64(uint64_t* a, int64_t n, gg_rng* r) {
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = (int64_t)rng_below(r, (uint64_t)(i + 1));
    uint64_t t = a[i]; a[i] = a[j]; a[j] = t;
  }
}

static void keys_to_edges(const uint64_t* keys, int64_t m, int64_t nL, int32_t* out) {
  for (int64_t i = 0; i < m; ++i) {
    out[2 * i] = (int32_t)(keys[i] / (uint64_t)nL);
    out[2 * i + 1] = (int32_t)(keys[i] % (uint64_t)nL);
  }
}

/* Pareto expected-degree weights: w = (1-q)^(-1/(gamma-1)), scaled so that
 * sum(w) = target and capped at `cap` (scale and cap are repeated until the
 * sum settles). */
static void chung_lu_weights(double* w, int64_t n, double gamma, double target, double cap, gg_rng* r) {
  double a = 1.0 / (gamma - 1.0);
  for (int64_t i = 0; i < n; ++i) w[i] = pow(1.0 - rng_double(r), -a);
  for (int it = 0; it < 200; ++it) {
    double s = 0;
    for (int64_t i = 0; i < n; ++i) s += w[i];
    double f = target / s;
    if (fabs(f - 1.0) < 1e-12) break;
    for (int64_t i = 0; i < n; ++i) { w[i] *= f; if (w[i] > cap) w[i] = cap; }
  }
}

/* ------------------------------------------------------------- public API */

/* m distinct cells of the nU x nL grid, uniformly without replacement. */
int64_t gg_uniform(uint64_t seed, int64_t nU, int64_t nL, int64_t m, int32_t* out) {
  if (nU <= 0 || nL <= 0 || m < 0 || m > nU * nL) return -1;
  gg_rng r; rng_seed(&r, seed);
  gg_pairdist d = {NULL, NULL, nU, nL};
  uint64_t* set = NULL;
  int64_t got = collect_pairs(&d, &r, m, NULL, 0, &set, 0);
  if (got != m) { free(set); return -2; }
  shuffle_u64(set, m, &r);
  keys_to_edges(set, m, nL, out);
  free(set);
  return m;
}

/*
 * Bipartite Chung-Lu graph with Pareto expected degrees (pdf exponent
 * gammaU / gammaL, cap `cap`), plus `nblocks` planted bicliques of
 * block x block vertices on disjoint random vertex sets, each cell kept with
 * probability `density`.  Planted edges count toward m.
 */
int64_t gg_chung_lu(uint64_t seed, int64_t nU, int64_t nL, int64_t m, double gammaU, double gammaL,
                    double cap, int64_t nblocks, int64_t block, double density, int32_t* out) {
  if (nU <= 0 || nL <= 0 || m < 0 || m > nU * nL) return -1;
  if (nblocks * block > nU || nblocks * block > nL) return -1;
  gg_rng r; rng_seed(&r, seed);
  /* planted blocks first */
  int64_t np = 0;
  uint64_t* planted = NULL;
  if (nblocks > 0 && block > 0) {
    int32_t* pu = (int32_t*)malloc(sizeof(int32_t) * (size_t)nU);
    int32_t* pl = (int32_t*)malloc(sizeof(int32_t) * (size_t)nL);
    planted = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(nblocks * block * block));
    if (!pu || !pl || !planted) return -3;
    for (int64_t i = 0; i < nU; ++i) pu[i] = (int32_t)i;
    for (int64_t i = 0; i < nL; ++i) pl[i] = (int32_t)i;
    int64_t take = nblocks * block;
    for (int64_t i = 0; i < take; ++i) { /* partial Fisher-Yates */
      int64_t j = i + (int64_t)rng_below(&r, (uint64_t)(nU - i));
      int32_t t = pu[i]; pu[i] = pu[j]; pu[j] = t;
    }
    for (int64_t i = 0; i < take; ++i) {
      int64_t j = i + (int64_t)rng_below(&r, (uint64_t)(nL - i));
      int32_t t = pl[i]; pl[i] = pl[j]; pl[j] = t;
    }
    for (int64_t b = 0; b < nblocks; ++b)
      for (int64_t i = 0; i < block; ++i)
        for (int64_t j = 0; j < block; ++j)
          if (rng_double(&r) < density)
            planted[np++] = (uint64_t)pu[b * block + i] * (uint64_t)nL + (uint64_t)pl[b * block + j];
    free(pu); free(pl);
    if (np > m) return -4;
    sort_u64(planted, np, bits_for((uint64_t)nU * (uint64_t)nL));
    np = unique_sorted(planted, np);
  }
  double target = (double)(m - np);
  double* wu = (double*)malloc(sizeof(double) * (size_t)nU);
  double* wl = (double*)malloc(sizeof(double) * (size_t)nL);
  if (!wu || !wl) return -3;
  chung_lu_weights(wu, nU, gammaU, target > 0 ? target : 1.0, cap, &r);
  chung_lu_weights(wl, nL, gammaL, target > 0 ? target : 1.0, cap, &r);
  gg_alias au, al;
  if (alias_build(&au, wu, nU) || alias_build(&al, wl, nL)) return -3;
  free(wu); free(wl);
  gg_pairdist d = {&au, &al, nU, nL};
  uint64_t* set = NULL;
  int64_t got = collect_pairs(&d, &r, m - np, planted, np, &set, 64);
  alias_free(&au); alias_free(&al);
  if (got != m - np) { free(set); free(planted); return -2; }
  uint64_t* all = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(m > 0 ? m : 1));
  if (!all) return -3;
  if (np) memcpy(all, planted, sizeof(uint64_t) * (size_t)np);
  if (m - np) memcpy(all + np, set, sizeof(uint64_t) * (size_t)(m - np));
  free(set); free(planted);
  shuffle_u64(all, m, &r);
  keys_to_edges(all, m, nL, out);
  free(all);
  return m;
}

/* Draws `count` doubles in [0,1) from the stream of `seed` (for host-side
 * parameter schedules that must match the C stream exactly). */
void gg_doubles(uint64_t seed, int64_t count, double* out) {
  gg_rng r; rng_seed(&r, seed);
  for (int64_t i = 0; i < count; ++i) out[i] = rng_double(&r);
}

/* Mixes a configuration seed and a sub-index into one seed (SplitMix64). */
uint64_t gg_subseed(uint64_t seed, uint64_t index) {
  uint64_t x = seed * 0x9E3779B97F4A7C15ull + index;
  splitmix64(&x);
  return splitmix64(&x);
}
