/*
 * Sequential decoder, validator and seek of the CPU oracle (test
 * infrastructure only).
 *
 * Decoding follows the plain definition: blocks in increasing order; for
 * each block the three streams (literals, lengths, absolute offsets) are
 * entropy-decoded, then each sequence k appends L_k literals and copies M_k
 * bytes one at a time from absolute position O_k (paper Section 2: the
 * back-reference already names a position in the decompressed output, so
 * no window or running distance is involved).  Every structural fact the
 * archive stores (dependency lists, levels, depth) is recomputed from the
 * tokens and compared.  A seek of [lo, hi) is decode_all(A)[lo:hi]; the
 * closure helper lists the blocks the paper's isolated seek needs (Section 3:
 * with absolute offsets a block needs only the earlier blocks its matches
 * copy from, not the whole prefix).
 */
#include <omp.h>
#include <stdlib.h>
#include <string.h>
#include "internal.h"

typedef struct {
  const uint8_t* a;
  uint64_t len, n;
  uint32_t B, W, ow, nb, depth, n_deps, max_level;
  uint64_t deps_at, pay_at;
} hdr_t;

static int parse_header(const uint8_t* a, uint64_t len, hdr_t* h) {
  if (!a) return orc_fail(ORC_E_ARG, "null archive");
  if (len < ORC_HDR) return orc_fail(ORC_E_CORRUPT, "archive shorter than its header");
  if (rd32(a) != ORC_MAGIC) return orc_fail(ORC_E_CORRUPT, "bad magic");
  if (rd16(a + 4) != ORC_VERSION) return orc_fail(ORC_E_CORRUPT, "unknown version %u", rd16(a + 4));
  h->a = a;
  h->len = len;
  h->B = rd32(a + 8);
  h->W = rd16(a + 12);
  h->ow = a[15];
  h->n = rd64(a + 16);
  h->nb = rd32(a + 24);
  h->depth = rd32(a + 28);
  h->n_deps = rd32(a + 36);
  h->max_level = rd32(a + 32);
  if (a[14] != ORC_PROB_BITS) return orc_fail(ORC_E_CORRUPT, "probability bits %u, expected 12", a[14]);
  if (h->B < 1 || h->B > (1u << 24)) return orc_fail(ORC_E_CORRUPT, "block size %u", h->B);
  if (h->W < 1 || h->W > 64) return orc_fail(ORC_E_CORRUPT, "interleave %u", h->W);
  if (h->ow != 4 && h->ow != 8) return orc_fail(ORC_E_CORRUPT, "offset width %u", h->ow);
  if (h->ow == 4 && h->n > (1ull << 32)) return orc_fail(ORC_E_CORRUPT, "4-byte offsets for a >4 GiB output");
  uint64_t nb = h->n ? (h->n - 1) / h->B + 1 : 0;
  if (nb != h->nb) return orc_fail(ORC_E_CORRUPT, "block count %u, expected %llu", h->nb, (unsigned long long)nb);
  if (rd64(a + 40) != ORC_HDR) return orc_fail(ORC_E_CORRUPT, "block table not right after the header");
  h->deps_at = ORC_HDR + (uint64_t)ORC_BLK * h->nb;
  h->pay_at = rd64(a + 48);
  if (h->deps_at + 4ull * h->n_deps > len || h->pay_at < h->deps_at + 4ull * h->n_deps || h->pay_at > len)
    return orc_fail(ORC_E_CORRUPT, "index overruns the archive");
  return ORC_OK;
}

/* Block b's table entry, checked against the archive bounds.  Returns the
 * dependency list position and count; levels are checked by the caller. */
typedef struct {
  uint64_t pay;
  uint32_t pay_len, n_seq, level, dep_off, dep_cnt;
} blk_t;

static int read_block(const hdr_t* h, uint32_t b, blk_t* e) {
  const uint8_t* p = h->a + ORC_HDR + (uint64_t)ORC_BLK * b;
  e->pay = rd64(p);
  e->pay_len = rd32(p + 8);
  e->n_seq = rd32(p + 12);
  e->level = rd32(p + 16);
  e->dep_off = rd32(p + 20);
  e->dep_cnt = rd32(p + 24);
  if (rd32(p + 28) != 0) return orc_fail(ORC_E_CORRUPT, "block %u: reserved field set", b);
  if (e->pay % 16 || e->pay < h->pay_at || e->pay + e->pay_len > h->len || e->pay_len < ORC_NSTREAM * ORC_SDESC)
    return orc_fail(ORC_E_CORRUPT, "block %u: payload outside the archive", b);
  if ((uint64_t)e->dep_off + e->dep_cnt > h->n_deps)
    return orc_fail(ORC_E_CORRUPT, "block %u: dependency list outside the index", b);
  const uint8_t* d = h->a + h->deps_at + 4ull * e->dep_off;
  for (uint32_t i = 0; i < e->dep_cnt; i++) {
    uint32_t v = rd32(d + 4 * i);
    if (v >= b) return orc_fail(ORC_E_CORRUPT, "block %u: dependency %u is not earlier", b, v);
    if (i && v <= rd32(d + 4 * (i - 1))) return orc_fail(ORC_E_CORRUPT, "block %u: dependencies not ascending", b);
  }
  return ORC_OK;
}

/* Decodes stream t of a block into out (n_sym bytes). */
static int decode_stream(const hdr_t* h, uint32_t b, const blk_t* e, int t, uint32_t want,
                         uint8_t* out) {
  const uint8_t* pl = h->a + e->pay;
  const uint8_t* d = pl + ORC_SDESC * t;
  uint8_t mode = d[0];
  uint32_t n_sym = rd32(d + 4), clen = rd32(d + 8), off = rd32(d + 12);
  if (d[1] || d[2] || d[3]) return orc_fail(ORC_E_CORRUPT, "block %u stream %d: padding set", b, t);
  if (n_sym != want) return orc_fail(ORC_E_CORRUPT, "block %u stream %d: %u symbols, expected %u", b, t, n_sym, want);
  if (off % 4 || off < ORC_NSTREAM * ORC_SDESC || (uint64_t)off + clen > e->pay_len)
    return orc_fail(ORC_E_CORRUPT, "block %u stream %d: data outside the payload", b, t);
  if (mode == 0) {
    if (clen != n_sym) return orc_fail(ORC_E_CORRUPT, "block %u stream %d: raw length mismatch", b, t);
    memcpy(out, pl + off, n_sym);
    return ORC_OK;
  }
  if (mode != 1) return orc_fail(ORC_E_CORRUPT, "block %u stream %d: unknown mode %u", b, t, mode);
  if (n_sym == 0) return orc_fail(ORC_E_CORRUPT, "block %u stream %d: empty rANS stream", b, t);
  uint16_t freq[256];
  int tsz = orc_table_read(pl + off, clen, freq);
  if (tsz < 0) return tsz;
  int rc = orc_rans_decode(pl + off + tsz, clen - (uint32_t)tsz, n_sym, h->W, freq, out);
  if (rc) return orc_fail(rc, "block %u stream %d: %s", b, t, orc_last_error());
  return ORC_OK;
}

static int cmp_u32(const void* x, const void* y) {
  uint32_t u = *(const uint32_t*)x, v = *(const uint32_t*)y;
  return u < v ? -1 : u > v;
}

/* Decodes block b into out (absolute positions); blocks before b that its
 * sources touch must already be present in out.  Also checks the stored
 * dependency list and level against the ones the tokens imply. */
static int decode_block(const hdr_t* h, uint32_t b, const uint32_t* levels, uint8_t* out,
                        uint32_t* level_out) {
  blk_t e;
  int rc = read_block(h, b, &e);
  if (rc) return rc;
  uint64_t s = (uint64_t)b * h->B, end = s + h->B < h->n ? s + h->B : h->n;
  uint64_t blen = end - s;
  if (e.n_seq == 0 || e.n_seq > blen) return orc_fail(ORC_E_CORRUPT, "block %u: %u sequences", b, e.n_seq);
  uint8_t* lens = (uint8_t*)malloc(4ull * e.n_seq);
  uint8_t* offs = (uint8_t*)malloc((uint64_t)h->ow * e.n_seq);
  uint8_t* lit = NULL;
  uint32_t* touched = NULL;
  uint32_t n_touch = 0;
  if (!lens || !offs) {
    rc = orc_fail(ORC_E_NOMEM, "out of memory");
    goto done;
  }
  if ((rc = decode_stream(h, b, &e, ORC_STREAM_LEN, 4 * e.n_seq, lens))) goto done;
  if ((rc = decode_stream(h, b, &e, ORC_STREAM_OFF, h->ow * e.n_seq, offs))) goto done;
  uint64_t nlit = 0, cover = 0;
  for (uint32_t k = 0; k < e.n_seq; k++) {
    nlit += rd16(lens + 4 * k);
    cover += rd16(lens + 4 * k) + rd16(lens + 4 * k + 2);
  }
  if (cover != blen)
    rc = orc_fail(ORC_E_CORRUPT, "block %u: sequences cover %llu of %llu bytes", b,
                  (unsigned long long)cover, (unsigned long long)blen);
  if (rc) goto done;
  lit = (uint8_t*)malloc(nlit ? nlit : 1);
  /* each match touches at most ceil(M/B)+1 earlier blocks */
  touched = (uint32_t*)malloc(sizeof(uint32_t) * (2 * (uint64_t)e.n_seq + blen / h->B + 2));
  if (!lit || !touched) {
    rc = orc_fail(ORC_E_NOMEM, "out of memory");
    goto done;
  }
  if ((rc = decode_stream(h, b, &e, ORC_STREAM_LIT, (uint32_t)nlit, lit))) goto done;
  /* expansion: literals, then byte-by-byte copies from absolute offsets */
  uint64_t pos = s, li = 0;
  for (uint32_t k = 0; k < e.n_seq; k++) {
    uint32_t L = rd16(lens + 4 * k), M = rd16(lens + 4 * k + 2);
    uint64_t O = h->ow == 4 ? rd32(offs + 4 * k) : rd64(offs + 8 * k);
    memcpy(out + pos, lit + li, L);
    pos += L;
    li += L;
    if (M == 0) {
      if (O != 0) {
        rc = orc_fail(ORC_E_CORRUPT, "block %u seq %u: offset without a match", b, k);
        goto done;
      }
      continue;
    }
    if (O >= pos) {
      rc = orc_fail(ORC_E_CORRUPT, "block %u seq %u: source %llu not before destination %llu", b, k,
                    (unsigned long long)O, (unsigned long long)pos);
      goto done;
    }
    for (uint32_t i = 0; i < M; i++) out[pos + i] = out[O + i];
    uint64_t src_end = O + M < s ? O + M : s;
    for (uint64_t q = O; q < src_end; q = (q / h->B + 1) * h->B) touched[n_touch++] = (uint32_t)(q / h->B);
    pos += M;
  }
  /* dependency list and level implied by the tokens */
  const uint8_t* d = h->a + h->deps_at + 4ull * e.dep_off;
  uint32_t cnt = 0, lv = 0;
  qsort(touched, n_touch, sizeof(uint32_t), cmp_u32);
  for (uint32_t i = 0; i < n_touch; i++) {
    uint32_t c = touched[i];
    if (i && touched[i - 1] == c) continue;
    if (cnt >= e.dep_cnt || rd32(d + 4 * cnt) != c) {
      rc = orc_fail(ORC_E_CORRUPT, "block %u: stored dependency list differs from the tokens", b);
      goto done;
    }
    cnt++;
    if (levels[c] + 1 > lv) lv = levels[c] + 1;
  }
  if (cnt != e.dep_cnt) {
    rc = orc_fail(ORC_E_CORRUPT, "block %u: stored dependency list differs from the tokens", b);
    goto done;
  }
  if (lv != e.level) {
    rc = orc_fail(ORC_E_CORRUPT, "block %u: stored level %u, tokens imply %u", b, e.level, lv);
    goto done;
  }
  *level_out = lv;
done:
  free(lens); free(offs); free(lit); free(touched);
  return rc;
}

/* Sequential decode of blocks [0, nb_upto) into out, with all checks. */
static int decode_prefix(const hdr_t* h, uint32_t nb_upto, uint8_t* out) {
  uint32_t* levels = (uint32_t*)malloc(sizeof(uint32_t) * (h->nb ? h->nb : 1));
  if (!levels) return orc_fail(ORC_E_NOMEM, "out of memory");
  int rc = ORC_OK;
  uint32_t maxlv = 0;
  for (uint32_t b = 0; b < nb_upto && !rc; b++) {
    rc = decode_block(h, b, levels, out, &levels[b]);
    if (!rc && levels[b] + 1 > maxlv) maxlv = levels[b] + 1;
  }
  if (!rc && nb_upto == h->nb && maxlv != h->depth)
    rc = orc_fail(ORC_E_CORRUPT, "stored depth %u, levels imply %u", h->depth, maxlv);
  if (!rc && h->max_level && maxlv > h->max_level)
    rc = orc_fail(ORC_E_CORRUPT, "a level reaches %u, above the stated cap %u", maxlv - 1, h->max_level - 1);
  free(levels);
  return rc;
}

int orc_info(const uint8_t* a, uint64_t len, uint64_t* n_total, uint32_t* block_size,
             uint32_t* n_blocks, uint32_t* depth, uint32_t* interleave) {
  hdr_t h;
  int rc = parse_header(a, len, &h);
  if (rc) return rc;
  if (n_total) *n_total = h.n;
  if (block_size) *block_size = h.B;
  if (n_blocks) *n_blocks = h.nb;
  if (depth) *depth = h.depth;
  if (interleave) *interleave = h.W;
  return ORC_OK;
}

int orc_decode(const uint8_t* a, uint64_t len, uint8_t* out, uint64_t cap) {
  hdr_t h;
  int rc = parse_header(a, len, &h);
  if (rc) return rc;
  if (cap < h.n) return orc_fail(ORC_E_NOSPACE, "output needs %llu bytes", (unsigned long long)h.n);
  if (h.n && !out) return orc_fail(ORC_E_ARG, "null output");
  rc = decode_prefix(&h, h.nb, out);
  if (!rc && orc_fnv1a64(out, h.n) != rd64(a + 56))
    rc = orc_fail(ORC_E_CORRUPT, "decoded bytes do not match the stored FNV-1a-64");
  return rc;
}

int orc_seek(const uint8_t* a, uint64_t len, uint64_t lo, uint64_t hi, uint8_t* out) {
  hdr_t h;
  int rc = parse_header(a, len, &h);
  if (rc) return rc;
  if (lo > hi) return orc_fail(ORC_E_ARG, "inverted range");
  if (hi > h.n) return orc_fail(ORC_E_RANGE, "range end %llu beyond %llu", (unsigned long long)hi,
                                (unsigned long long)h.n);
  if (lo == hi) return ORC_OK;
  if (!out) return orc_fail(ORC_E_ARG, "null output");
  uint32_t last = (uint32_t)((hi - 1) / h.B);
  uint64_t upto = ((uint64_t)last + 1) * h.B < h.n ? ((uint64_t)last + 1) * h.B : h.n;
  uint8_t* tmp = (uint8_t*)malloc(upto);
  if (!tmp) return orc_fail(ORC_E_NOMEM, "out of memory");
  rc = decode_prefix(&h, last + 1, tmp);
  if (!rc) memcpy(out, tmp + lo, hi - lo);
  free(tmp);
  return rc;
}

int orc_closure(const uint8_t* a, uint64_t len, uint64_t lo, uint64_t hi, uint8_t* need,
                uint32_t* count) {
  hdr_t h;
  int rc = parse_header(a, len, &h);
  if (rc) return rc;
  if (lo > hi) return orc_fail(ORC_E_ARG, "inverted range");
  if (hi > h.n) return orc_fail(ORC_E_RANGE, "range beyond the output");
  memset(need, 0, h.nb);
  uint32_t cnt = 0;
  if (lo == hi) {
    *count = 0;
    return ORC_OK;
  }
  uint32_t first = (uint32_t)(lo / h.B), last = (uint32_t)((hi - 1) / h.B);
  for (uint32_t b = first; b <= last; b++) need[b] = 1;
  /* dependencies are always earlier blocks, so one descending sweep closes
   * the set */
  for (uint32_t b = last + 1; b-- > 0;) {
    if (!need[b]) continue;
    cnt++;
    blk_t e;
    if ((rc = read_block(&h, b, &e))) return rc;
    const uint8_t* d = a + h.deps_at + 4ull * e.dep_off;
    for (uint32_t i = 0; i < e.dep_cnt; i++) need[rd32(d + 4 * i)] = 1;
  }
  *count = cnt;
  return ORC_OK;
}

int orc_block_facts(const uint8_t* a, uint64_t len, uint32_t* level, uint32_t* n_seq,
                    uint8_t* modes) {
  hdr_t h;
  int rc = parse_header(a, len, &h);
  if (rc) return rc;
  for (uint32_t b = 0; b < h.nb; b++) {
    blk_t e;
    if ((rc = read_block(&h, b, &e))) return rc;
    level[b] = e.level;
    n_seq[b] = e.n_seq;
    for (int t = 0; t < 3; t++) modes[3 * b + t] = a[e.pay + ORC_SDESC * t];
  }
  return ORC_OK;
}

int orc_block_tokens(const uint8_t* a, uint64_t len, uint32_t block, uint8_t* lit,
                     uint32_t* n_lit, uint32_t* Ls, uint32_t* Ms, uint64_t* Os, uint32_t* n_seq) {
  hdr_t h;
  int rc = parse_header(a, len, &h);
  if (rc) return rc;
  if (block >= h.nb) return orc_fail(ORC_E_RANGE, "no block %u", block);
  blk_t e;
  if ((rc = read_block(&h, block, &e))) return rc;
  uint64_t s = (uint64_t)block * h.B, blen = (s + h.B < h.n ? s + h.B : h.n) - s;
  if (e.n_seq == 0 || e.n_seq > blen) return orc_fail(ORC_E_CORRUPT, "block %u: %u sequences", block, e.n_seq);
  uint8_t* lens = (uint8_t*)malloc(4ull * e.n_seq);
  uint8_t* offs = (uint8_t*)malloc((uint64_t)h.ow * e.n_seq);
  if (!lens || !offs) {
    free(lens); free(offs);
    return orc_fail(ORC_E_NOMEM, "out of memory");
  }
  rc = decode_stream(&h, block, &e, ORC_STREAM_LEN, 4 * e.n_seq, lens);
  if (!rc) rc = decode_stream(&h, block, &e, ORC_STREAM_OFF, h.ow * e.n_seq, offs);
  uint32_t nl = 0;
  for (uint32_t k = 0; !rc && k < e.n_seq; k++) {
    Ls[k] = rd16(lens + 4 * k);
    Ms[k] = rd16(lens + 4 * k + 2);
    Os[k] = h.ow == 4 ? rd32(offs + 4 * k) : rd64(offs + 8 * k);
    nl += Ls[k];
  }
  if (!rc && nl > blen) rc = orc_fail(ORC_E_CORRUPT, "block %u: too many literals", block);
  if (!rc) rc = decode_stream(&h, block, &e, ORC_STREAM_LIT, nl, lit);
  free(lens); free(offs);
  if (!rc) {
    *n_lit = nl;
    *n_seq = e.n_seq;
  }
  return rc;
}

/* Whole-archive decode with the blocks of one dependency level decoded in
 * parallel (OpenMP), levels in increasing order: a block's dependencies all
 * sit at lower levels (Section 2: with absolute offsets a block can be
 * decoded as soon as the earlier blocks it copies from are decoded), so the
 * blocks of one level are independent.
 * Each block goes through the same decode_block as the sequential decoder.
 * This is the all-cores CPU baseline, not a second definition of decode: on
 * any error the sequential decoder is run to report it. */
int orc_decode_levels(const uint8_t* a, uint64_t len, uint8_t* out, uint64_t cap, int threads,
                      int* threads_used) {
  hdr_t h;
  int rc = parse_header(a, len, &h);
  if (rc) return rc;
  if (cap < h.n) return orc_fail(ORC_E_NOSPACE, "output needs %llu bytes", (unsigned long long)h.n);
  if (h.n && !out) return orc_fail(ORC_E_ARG, "null output");
  uint32_t nb = h.nb, depth = h.depth;
  uint32_t* stored = (uint32_t*)malloc(sizeof(uint32_t) * (nb ? nb : 1));
  uint32_t* levels = (uint32_t*)malloc(sizeof(uint32_t) * (nb ? nb : 1));
  uint32_t* order = (uint32_t*)malloc(sizeof(uint32_t) * (nb ? nb : 1));
  uint32_t* lstart = (uint32_t*)calloc((size_t)depth + 2, sizeof(uint32_t));
  if (!stored || !levels || !order || !lstart) {
    free(stored); free(levels); free(order); free(lstart);
    return orc_fail(ORC_E_NOMEM, "out of memory");
  }
  for (uint32_t b = 0; b < nb && !rc; b++) {
    blk_t e;
    rc = read_block(&h, b, &e);
    if (!rc && e.level >= depth) rc = orc_fail(ORC_E_CORRUPT, "block %u: level %u not below depth %u", b, e.level, depth);
    if (!rc) {
      stored[b] = e.level;
      lstart[e.level + 1]++;
    }
  }
  if (!rc) {
    for (uint32_t l = 0; l < depth; l++) lstart[l + 1] += lstart[l];
    uint32_t* fill = (uint32_t*)malloc(sizeof(uint32_t) * (depth ? depth : 1));
    if (!fill) rc = orc_fail(ORC_E_NOMEM, "out of memory");
    for (uint32_t l = 0; !rc && l < depth; l++) fill[l] = lstart[l];
    for (uint32_t b = 0; !rc && b < nb; b++) order[fill[stored[b]]++] = b;
    free(fill);
  }
  int used = 1;
  int failed = rc != 0;
  for (uint32_t l = 0; l < depth && !failed; l++) {
    const int64_t lo = lstart[l], hi = lstart[l + 1];
#pragma omp parallel num_threads(threads > 0 ? threads : omp_get_max_threads())
    {
#pragma omp single
      used = omp_get_num_threads();
#pragma omp for schedule(dynamic, 8) reduction(| : failed)
      for (int64_t j = lo; j < hi; j++) {
        uint32_t lv = 0;
        if (decode_block(&h, order[j], levels, out, &lv)) failed = 1;
        else levels[order[j]] = lv;
      }
    }
  }
  free(stored); free(levels); free(order); free(lstart);
  if (threads_used) *threads_used = used;
  if (failed) return orc_decode(a, len, out, cap);  /* reports the error */
  if (h.max_level && depth > h.max_level)
    return orc_fail(ORC_E_CORRUPT, "a level reaches %u, above the stated cap %u", depth - 1, h.max_level - 1);
  if (orc_fnv1a64(out, h.n) != rd64(a + 56))
    return orc_fail(ORC_E_CORRUPT, "decoded bytes do not match the stored FNV-1a-64");
  return ORC_OK;
}
