/*
 * Match layer encoder and archive writer of the CPU oracle (test
 * infrastructure only).
 *
 * Paper Section 2: every LZ77 back-reference is stored as an absolute
 * position in the decompressed output, found by a global match search, and
 * the output is cut into fixed-size blocks.  The search here is a plain hash
 * chain over every position of the input:
 *   - hash of X[p .. p+hash_len): h = sum X[p+i] * 0x01000193^(hash_len-1-i)
 *     (mod 2^32), bucket = (h * 0x9E3779B1 mod 2^32) >> (32 - hbits), with
 *     hbits = clamp(ceil(log2 n), 12, 27); prev[p] = the previous position
 *     with the same bucket;
 *   - blocks are parsed in order; at p the chain from prev[p] is walked most
 *     recent first for at most max_chain candidates; a candidate q scores
 *     the common prefix of X[q..] and X[p..], capped at the block end and at
 *     65535 (overlap with p is allowed: the copy is byte-sequential);
 *   - with max_level > 0 blocks are grouped in epochs of 64 (E epochs in
 *     all), and epochs in units of c = max(1, floor(E / 64)); a block of
 *     epoch e may take sources only from itself and from blocks of earlier
 *     epochs whose level is below
 *         lambda(e) = min(max_level - 1, floor(log2(floor(e / c) + 1)),
 *                         max(1, floor(log2(floor(E / c) + 1)) - 1))
 *     ("visible" blocks), so every level stays below max_level and the
 *     levels grow geometrically in size from c epochs (the last level holds
 *     at least half of the epochs).  Chain candidates in invisible blocks are passed over
 *     without being counted (at most 8 * max_chain chain steps in all), and a
 *     counted candidate is cut where its source first enters an invisible
 *     block;
 *   - the longest candidate wins, ties to the first found (most recent);
 *     it is taken if it reaches min_match, else p is a literal.
 * The parse is encoder policy; any legal parse decodes to the same bytes.
 */
#include <stdlib.h>
#include <string.h>
#include "internal.h"

#define NONE UINT64_MAX

typedef struct {
  uint32_t *L, *M;
  uint64_t* O;
  uint64_t n, cap;
} seqvec;

static int seq_push(seqvec* v, uint32_t L, uint32_t M, uint64_t O) {
  if (v->n == v->cap) {
    uint64_t c = v->cap ? v->cap * 2 : 1024;
    uint32_t* nL = (uint32_t*)realloc(v->L, c * sizeof(uint32_t));
    if (!nL) return ORC_E_NOMEM;
    v->L = nL;
    uint32_t* nM = (uint32_t*)realloc(v->M, c * sizeof(uint32_t));
    if (!nM) return ORC_E_NOMEM;
    v->M = nM;
    uint64_t* nO = (uint64_t*)realloc(v->O, c * sizeof(uint64_t));
    if (!nO) return ORC_E_NOMEM;
    v->O = nO;
    v->cap = c;
  }
  v->L[v->n] = L;
  v->M[v->n] = M;
  v->O[v->n] = O;
  v->n++;
  return ORC_OK;
}

/* Emit a run of `lits` pending literals followed by a match (M may be 0).
 * Runs longer than 65535 are split into literal-only sequences. */
static int emit(seqvec* v, uint64_t lits, uint32_t M, uint64_t O) {
  while (lits > 65535) {
    if (seq_push(v, 65535, 0, 0)) return ORC_E_NOMEM;
    lits -= 65535;
  }
  return seq_push(v, (uint32_t)lits, M, O);
}

static uint32_t hash_bits_for(uint64_t n) {
  uint32_t b = 0;
  while (b < 64 && (1ull << b) < n) b++;
  if (b < 12) b = 12;
  if (b > 27) b = 27;
  return b;
}

/* ---- per-block dependency sets and levels (format definition) ---- */
/* deps(b) = { floor(q / B) : q in [O, min(O + M, b*B)), M > 0 }, sorted. */
static int cmp_u32(const void* a, const void* b) {
  uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
  return x < y ? -1 : x > y;
}

static int block_deps(uint32_t b, uint64_t B, const uint32_t* M, const uint64_t* O,
                      uint32_t nseq, uint32_t** out, uint32_t* cnt) {
  uint32_t n = 0, cap = 16;
  uint32_t* d = (uint32_t*)malloc(sizeof(uint32_t) * cap);
  if (!d) return ORC_E_NOMEM;
  uint64_t bs = (uint64_t)b * B;
  for (uint32_t k = 0; k < nseq; k++) {
    if (M[k] == 0) continue;
    uint64_t lo = O[k], hi = O[k] + M[k];
    if (hi > bs) hi = bs;
    for (uint64_t q = lo; q < hi; q = (q / B + 1) * B) {
      if (n == cap) {
        cap *= 2;
        uint32_t* nd = (uint32_t*)realloc(d, sizeof(uint32_t) * cap);
        if (!nd) {
          free(d);
          return ORC_E_NOMEM;
        }
        d = nd;
      }
      d[n++] = (uint32_t)(q / B);
    }
  }
  qsort(d, n, sizeof(uint32_t), cmp_u32);
  uint32_t u = 0;
  for (uint32_t i = 0; i < n; i++)
    if (u == 0 || d[u - 1] != d[i]) d[u++] = d[i];
  *out = d;
  *cnt = u;
  return ORC_OK;
}

/* ---- stream encoding ---- */
typedef struct {
  uint8_t mode;
  uint32_t n_sym, comp_len;
  uint8_t* data; /* comp_len bytes, malloc'd */
} enc_stream;

static int encode_stream(const uint8_t* sym, uint32_t n, uint32_t W, uint32_t policy,
                         enc_stream* es) {
  es->n_sym = n;
  es->mode = 0;
  es->comp_len = n;
  es->data = (uint8_t*)malloc(n ? n : 1);
  if (!es->data) return ORC_E_NOMEM;
  memcpy(es->data, sym, n);
  if (n == 0 || policy == ORC_MODE_RAW) return ORC_OK;
  uint64_t counts[256] = {0};
  for (uint32_t i = 0; i < n; i++) counts[sym[i]]++;
  uint16_t freq[256];
  int rc = orc_normalize(counts, freq);
  if (rc) return rc;
  uint32_t tsz = orc_table_size(freq);
  uint32_t cap = tsz + 4 * W + 2 * n;
  uint8_t* buf = (uint8_t*)malloc(cap);
  if (!buf) return ORC_E_NOMEM;
  orc_table_write(freq, buf);
  uint32_t body = 0;
  rc = orc_rans_encode(sym, n, W, freq, buf + tsz, cap - tsz, &body);
  if (rc) {
    free(buf);
    return rc;
  }
  if (policy == ORC_MODE_RANS || tsz + body < n) {
    free(es->data);
    es->data = buf;
    es->mode = 1;
    es->comp_len = tsz + body;
  } else {
    free(buf);
  }
  return ORC_OK;
}

static uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

/* ---- archive assembly from a parse ---- */
static int assemble(const uint8_t* x, uint64_t n, uint32_t B, uint32_t W, uint32_t flags,
                    uint32_t max_level, const uint32_t* seq_count, const uint32_t* L,
                    const uint32_t* M, const uint64_t* O, uint8_t** out, uint64_t* out_len) {
  uint32_t policy = flags & 3;
  uint64_t nb64 = n ? (n + B - 1) / B : 0;
  if (nb64 > 0xFFFFFFFFull) return orc_fail(ORC_E_ARG, "too many blocks");
  uint32_t nb = (uint32_t)nb64;
  /* offsets take 8 bytes once a position can exceed 32 bits, or on request */
  uint32_t ow = (n <= (1ull << 32) && !(flags & ORC_WIDE_OFFSETS)) ? 4 : 8;
  uint32_t *level = NULL, **deps = NULL, *dcnt = NULL;
  enc_stream* st = NULL;
  uint64_t* seq0 = NULL;
  uint8_t* buf = NULL;
  int rc = ORC_OK;
  level = (uint32_t*)calloc(nb ? nb : 1, sizeof(uint32_t));
  deps = (uint32_t**)calloc(nb ? nb : 1, sizeof(uint32_t*));
  dcnt = (uint32_t*)calloc(nb ? nb : 1, sizeof(uint32_t));
  st = (enc_stream*)calloc((size_t)(nb ? nb : 1) * 3, sizeof(enc_stream));
  seq0 = (uint64_t*)calloc((size_t)nb + 1, sizeof(uint64_t));
  if (!level || !deps || !dcnt || !st || !seq0) {
    rc = orc_fail(ORC_E_NOMEM, "assemble: out of memory");
    goto done;
  }
  for (uint32_t b = 0; b < nb; b++) seq0[b + 1] = seq0[b] + seq_count[b];
  /* check the parse reproduces x, then compute deps, levels and streams */
  uint64_t n_deps = 0;
  uint32_t depth = 0;
  for (uint32_t b = 0; b < nb; b++) {
    uint64_t s = (uint64_t)b * B, e = s + B < n ? s + B : n, p = s;
    uint64_t k0 = seq0[b], kn = seq_count[b];
    uint64_t nlit = 0;
    for (uint64_t k = k0; k < k0 + kn; k++) {
      if (L[k] > 65535 || M[k] > 65535) {
        rc = orc_fail(ORC_E_ARG, "block %u: length above 65535", b);
        goto done;
      }
      p += L[k];
      nlit += L[k];
      if (M[k]) {
        if (O[k] >= p || p + M[k] > e) {
          rc = orc_fail(ORC_E_ARG, "block %u seq %llu: bad match", b, (unsigned long long)(k - k0));
          goto done;
        }
        for (uint32_t i = 0; i < M[k]; i++)
          if (x[O[k] + i] != x[p + i]) {
            rc = orc_fail(ORC_E_ARG, "block %u seq %llu: match bytes differ", b,
                          (unsigned long long)(k - k0));
            goto done;
          }
      } else if (O[k] != 0) {
        rc = orc_fail(ORC_E_ARG, "block %u: offset without match", b);
        goto done;
      }
      p += M[k];
      if (p > e) {
        rc = orc_fail(ORC_E_ARG, "block %u: sequences overrun the block", b);
        goto done;
      }
    }
    if (p != e) {
      rc = orc_fail(ORC_E_ARG, "block %u: sequences cover %llu of %llu bytes", b,
                    (unsigned long long)(p - s), (unsigned long long)(e - s));
      goto done;
    }
    rc = block_deps(b, B, M + k0, O + k0, (uint32_t)kn, &deps[b], &dcnt[b]);
    if (rc) goto done;
    uint32_t lv = 0;
    for (uint32_t i = 0; i < dcnt[b]; i++)
      if (level[deps[b][i]] + 1 > lv) lv = level[deps[b][i]] + 1;
    level[b] = lv;
    if (lv + 1 > depth) depth = lv + 1;
    n_deps += dcnt[b];
    /* the three streams of the block */
    uint8_t* lit = (uint8_t*)malloc(nlit ? nlit : 1);
    uint8_t* lens = (uint8_t*)malloc(kn ? 4 * kn : 1);
    uint8_t* offs = (uint8_t*)malloc(kn ? ow * kn : 1);
    if (!lit || !lens || !offs) {
      free(lit); free(lens); free(offs);
      rc = orc_fail(ORC_E_NOMEM, "assemble: out of memory");
      goto done;
    }
    uint64_t q = s, li = 0;
    for (uint64_t k = 0; k < kn; k++) {
      memcpy(lit + li, x + q, L[k0 + k]);
      li += L[k0 + k];
      q += L[k0 + k] + M[k0 + k];
      wr16(lens + 4 * k, (uint16_t)L[k0 + k]);
      wr16(lens + 4 * k + 2, (uint16_t)M[k0 + k]);
      for (uint32_t i = 0; i < ow; i++) offs[ow * k + i] = (uint8_t)(O[k0 + k] >> (8 * i));
    }
    int r1 = encode_stream(lit, (uint32_t)nlit, W, policy, &st[3 * b + 0]);
    int r2 = r1 ? r1 : encode_stream(lens, (uint32_t)(4 * kn), W, policy, &st[3 * b + 1]);
    int r3 = r2 ? r2 : encode_stream(offs, (uint32_t)(ow * kn), W, policy, &st[3 * b + 2]);
    free(lit); free(lens); free(offs);
    if (r3) {
      rc = orc_fail(r3, "assemble: stream encoding failed: %s", orc_last_error());
      goto done;
    }
  }
  if (n_deps > 0xFFFFFFFFull) {
    rc = orc_fail(ORC_E_ARG, "too many dependency entries");
    goto done;
  }
  /* sizes: header, block table, deps, then 16-aligned block payloads */
  uint64_t deps_at = ORC_HDR + (uint64_t)ORC_BLK * nb;
  uint64_t pay_at = align_up(deps_at + 4 * n_deps, 16);
  uint64_t total = pay_at;
  for (uint32_t b = 0; b < nb; b++) {
    uint64_t sz = ORC_NSTREAM * ORC_SDESC;
    for (int t = 0; t < 3; t++) sz = align_up(sz, 4) + st[3 * b + t].comp_len;
    total = align_up(total, 16) + sz;
  }
  buf = (uint8_t*)calloc(total ? total : 1, 1);
  if (!buf) {
    rc = orc_fail(ORC_E_NOMEM, "assemble: out of memory");
    goto done;
  }
  wr32(buf + 0, ORC_MAGIC);
  wr16(buf + 4, ORC_VERSION);
  wr16(buf + 6, 0);
  wr32(buf + 8, B);
  wr16(buf + 12, (uint16_t)W);
  buf[14] = ORC_PROB_BITS;
  buf[15] = (uint8_t)ow;
  wr64(buf + 16, n);
  wr32(buf + 24, nb);
  wr32(buf + 28, depth);
  wr32(buf + 32, max_level);
  wr32(buf + 36, (uint32_t)n_deps);
  wr64(buf + 40, ORC_HDR);
  wr64(buf + 48, pay_at);
  wr64(buf + 56, orc_fnv1a64(x, n));
  uint64_t at = pay_at, di = 0;
  for (uint32_t b = 0; b < nb; b++) {
    at = align_up(at, 16);
    uint8_t* be = buf + ORC_HDR + (uint64_t)ORC_BLK * b;
    uint8_t* pl = buf + at;
    uint64_t off = ORC_NSTREAM * ORC_SDESC;
    for (int t = 0; t < 3; t++) {
      enc_stream* es = &st[3 * b + t];
      off = align_up(off, 4);
      uint8_t* d = pl + ORC_SDESC * t;
      d[0] = es->mode;
      wr32(d + 4, es->n_sym);
      wr32(d + 8, es->comp_len);
      wr32(d + 12, (uint32_t)off);
      memcpy(pl + off, es->data, es->comp_len);
      off += es->comp_len;
    }
    wr64(be + 0, at);
    wr32(be + 8, (uint32_t)off);
    wr32(be + 12, seq_count[b]);
    wr32(be + 16, level[b]);
    wr32(be + 20, (uint32_t)di);
    wr32(be + 24, dcnt[b]);
    wr32(be + 28, 0);
    for (uint32_t i = 0; i < dcnt[b]; i++) wr32(buf + deps_at + 4 * (di + i), deps[b][i]);
    di += dcnt[b];
    at += off;
  }
  *out = buf;
  *out_len = total;
  buf = NULL;
done:
  free(buf);
  if (deps)
    for (uint32_t b = 0; b < nb; b++) free(deps[b]);
  if (st)
    for (uint64_t i = 0; i < (uint64_t)nb * 3; i++) free(st[i].data);
  free(deps); free(dcnt); free(level); free(st); free(seq0);
  return rc;
}

static int check_params(uint64_t n, const orc_params* p) {
  if (!p) return orc_fail(ORC_E_ARG, "null params");
  if (p->block_size < 1 || p->block_size > (1u << 24)) return orc_fail(ORC_E_ARG, "block_size outside 1..2^24");
  if (p->interleave < 1 || p->interleave > 64) return orc_fail(ORC_E_ARG, "interleave outside 1..64");
  if (p->hash_len < 1 || p->hash_len > 64) return orc_fail(ORC_E_ARG, "hash_len outside 1..64");
  if (p->min_match < p->hash_len) return orc_fail(ORC_E_ARG, "min_match below hash_len");
  if ((p->flags & 3) == 3) return orc_fail(ORC_E_ARG, "bad stream-mode policy");
  if (p->flags & ~7u) return orc_fail(ORC_E_ARG, "unknown flag bits");
  (void)n;
  return ORC_OK;
}

int orc_encode_bound(uint64_t n, const orc_params* p, uint64_t* bound) {
  int rc = check_params(n, p);
  if (rc) return rc;
  uint64_t B = p->block_size, nb = n ? (n + B - 1) / B : 0;
  uint64_t W = p->interleave, ow = (n <= (1ull << 32) && !(p->flags & ORC_WIDE_OFFSETS)) ? 4 : 8;
  uint64_t total = ORC_HDR + ORC_BLK * nb + 16;
  for (uint64_t b = 0; b < nb; b++) {
    uint64_t len = (b + 1) * B <= n ? B : n - b * B;
    uint64_t nseq = len / p->min_match + len / 65535 + 2;
    if (nseq > len) nseq = len;
    uint64_t dep = 2 * nseq + 1;
    if (dep > b) dep = b;
    uint64_t syms[3] = {len, 4 * nseq, ow * nseq};
    uint64_t sz = 16 + ORC_NSTREAM * ORC_SDESC + 4 * dep;
    for (int t = 0; t < 3; t++)
      sz += 3 + ((p->flags & 3) == ORC_MODE_RANS ? 544 + 4 * W + 2 * syms[t] : syms[t]);
    total += sz;
  }
  *bound = total;
  return ORC_OK;
}

/* floor(log2(v)) for v >= 1 */
static uint32_t ilog2(uint64_t v) {
  uint32_t r = 0;
  while (v >>= 1) r++;
  return r;
}

/* Level budget of epoch e of E under cap max_level: blocks of the epoch see
 * only earlier-epoch blocks whose level is below this value. */
static uint32_t level_budget(uint64_t e, uint64_t E, uint32_t max_level) {
  uint64_t c = E / 64 > 1 ? E / 64 : 1;
  uint32_t lam = ilog2(e / c + 1);
  uint32_t top = ilog2(E / c + 1);
  top = top >= 2 ? top - 1 : 1;
  if (lam > top) lam = top;
  if (lam > max_level - 1) lam = max_level - 1;
  return lam;
}

int orc_encode(const uint8_t* src, uint64_t n, const orc_params* p, uint8_t* dst,
               uint64_t cap, uint64_t* out_len) {
  int rc = check_params(n, p);
  if (rc) return rc;
  if ((!src && n) || !out_len) return orc_fail(ORC_E_ARG, "null pointer");
  uint64_t B = p->block_size, nb = n ? (n + B - 1) / B : 0;
  if (nb > 0xFFFFFFFFull) return orc_fail(ORC_E_ARG, "too many blocks");
  uint32_t hbits = hash_bits_for(n);
  uint64_t* head = (uint64_t*)malloc(sizeof(uint64_t) << hbits);
  uint64_t* prev = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
  uint32_t* level = (uint32_t*)calloc(nb ? nb : 1, sizeof(uint32_t));
  uint32_t* seq_count = (uint32_t*)calloc(nb ? nb : 1, sizeof(uint32_t));
  seqvec v = {0};
  uint8_t* arch = NULL;
  uint64_t alen = 0;
  if (!head || !prev || !level || !seq_count) {
    rc = orc_fail(ORC_E_NOMEM, "encode: out of memory");
    goto done;
  }
  for (uint64_t i = 0; i < (1ull << hbits); i++) head[i] = NONE;
  /* insert every position whose hash window fits, in increasing order */
  for (uint64_t q = 0; q < n; q++) {
    prev[q] = NONE;
    if (q + p->hash_len > n) continue;
    uint32_t h = 0;
    for (uint32_t i = 0; i < p->hash_len; i++) h = h * 0x01000193u + src[q + i];
    uint32_t bucket = (uint32_t)((h * 0x9E3779B1u) >> (32 - hbits));
    prev[q] = head[bucket];
    head[bucket] = q;
  }
  for (uint64_t b = 0; b < nb; b++) {
    uint64_t s = b * B, e = s + B < n ? s + B : n, pos = s, lit0 = s;
    uint64_t first = v.n;
    while (pos < e) {
      uint64_t best = 0, bestq = 0;
      if (pos + p->hash_len <= n && e - pos >= p->min_match) {
        uint64_t q = prev[pos];
        uint32_t cand = 0, steps = 0;
        uint64_t lim = e - pos < 65535 ? e - pos : 65535;
        /* first byte of this block's epoch: earlier blocks of the epoch are invisible */
        uint64_t epoch0 = p->max_level > 0 ? (b / 64) * 64 * B : s;
        uint32_t lam = p->max_level > 0 ? level_budget(b / 64, (nb + 63) / 64, p->max_level) : 0;
        for (; q != NONE && cand < p->max_chain && steps < 8 * p->max_chain; steps++, q = prev[q]) {
          if (p->max_level > 0 && q < s && (q >= epoch0 || level[q / B] >= lam))
            continue; /* starts in an invisible block: passed over, not counted */
          cand++;
          uint64_t len = 0;
          while (len < lim && src[q + len] == src[pos + len]) len++;
          if (p->max_level > 0) {
            /* cut where the source first enters an invisible block */
            uint64_t end = q + len < s ? q + len : s;
            for (uint64_t c = q / B; c * B < end; c++)
              if (c * B >= epoch0 || level[c] >= lam) {
                len = c * B > q ? c * B - q : 0;
                break;
              }
          }
          if (len > best) {
            best = len;
            bestq = q;
          }
        }
      }
      if (best >= p->min_match) {
        if (emit(&v, pos - lit0, (uint32_t)best, bestq)) {
          rc = orc_fail(ORC_E_NOMEM, "encode: out of memory");
          goto done;
        }
        pos += best;
        lit0 = pos;
      } else {
        pos++;
      }
    }
    if (lit0 < e && emit(&v, e - lit0, 0, 0)) {
      rc = orc_fail(ORC_E_NOMEM, "encode: out of memory");
      goto done;
    }
    seq_count[b] = (uint32_t)(v.n - first);
    /* level of this block, needed by the cap when parsing later blocks */
    uint32_t* d = NULL;
    uint32_t dc = 0;
    rc = block_deps((uint32_t)b, B, v.M + first, v.O + first, seq_count[b], &d, &dc);
    if (rc) {
      rc = orc_fail(rc, "encode: out of memory");
      goto done;
    }
    uint32_t lv = 0;
    for (uint32_t i = 0; i < dc; i++)
      if (level[d[i]] + 1 > lv) lv = level[d[i]] + 1;
    level[b] = lv;
    free(d);
  }
  free(head);
  head = NULL;
  free(prev);
  prev = NULL;
  rc = assemble(src, n, p->block_size, p->interleave, p->flags, p->max_level, seq_count,
                v.L, v.M, v.O, &arch, &alen);
  if (rc) goto done;
  *out_len = alen;
  if (alen > cap || !dst) {
    rc = orc_fail(ORC_E_NOSPACE, "encode: archive needs %llu bytes", (unsigned long long)alen);
    goto done;
  }
  memcpy(dst, arch, alen);
done:
  free(arch); free(head); free(prev); free(level); free(seq_count);
  free(v.L); free(v.M); free(v.O);
  return rc;
}

int orc_assemble(const uint8_t* x, uint64_t n, uint32_t block_size, uint32_t interleave,
                 uint32_t flags, const uint32_t* seq_count, const uint32_t* L,
                 const uint32_t* M, const uint64_t* O, uint8_t* dst, uint64_t cap,
                 uint64_t* out_len) {
  if (block_size < 1 || block_size > (1u << 24) || interleave < 1 || interleave > 64 ||
      (flags & 3) == 3 || (flags & ~7u) || !out_len || (!x && n))
    return orc_fail(ORC_E_ARG, "assemble: bad arguments");
  uint8_t* arch = NULL;
  uint64_t alen = 0;
  int rc = assemble(x, n, block_size, interleave, flags, 0, seq_count, L, M, O, &arch, &alen);
  if (rc) return rc;
  *out_len = alen;
  if (alen > cap || !dst) {
    free(arch);
    return orc_fail(ORC_E_NOSPACE, "assemble: archive needs %llu bytes", (unsigned long long)alen);
  }
  memcpy(dst, arch, alen);
  free(arch);
  return ORC_OK;
}
