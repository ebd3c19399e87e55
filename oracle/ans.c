/*
 * Entropy layer of the CPU oracle (test infrastructure only).
 *
 * rANS (Duda's range variant of asymmetric numeral systems) over a byte
 * alphabet with 12-bit probabilities (M = 4096), one 32-bit state per lane,
 * state interval [L, 2^32) with L = 2^16 and 16-bit renormalisation words,
 * so that a symbol renormalises at most once.  W states are interleaved in
 * Giesen's manner: symbol i belongs to lane i mod W.  The paper uses an
 * off-the-shelf GPU ANS library as its entropy layer and does not fix these
 * parameters (Sections 1 and 9); the 32-way / 12-bit / u32 choice is the
 * configuration of the smallest workload, and the 16-bit renormalisation
 * unit is this codec's reading.
 *
 * Encoder, for i = n-1 down to 0, j = i mod W, s = sym[i]:
 *     if x_j >= 2^20 * f_s: emit the low 16 bits of x_j, x_j >>= 16
 *     x_j = floor(x_j / f_s) * M + (x_j mod f_s) + cum_s
 * then the stream is the W final states followed by the emitted words in
 * reverse order.  Decoder, for i = 0..n-1 (lane j = i mod W):
 *     slot = x_j mod M; s = symbol whose [cum_s, cum_s + f_s) holds slot
 *     x_j = f_s * (x_j >> 12) + slot - cum_s
 *     if x_j < L: x_j = (x_j << 16) | next word
 * and every final state must be L again.
 */
#include <stdlib.h>
#include <string.h>
#include "internal.h"

int orc_normalize(const uint64_t* counts, uint16_t* freq) {
  uint64_t n = 0;
  for (int s = 0; s < 256; s++) n += counts[s];
  if (n == 0) return orc_fail(ORC_E_ARG, "normalize: no symbols");
  uint32_t f[256];
  int64_t sum = 0;
  for (int s = 0; s < 256; s++) {
    if (counts[s] == 0) {
      f[s] = 0;
      continue;
    }
    uint64_t v = (counts[s] * (uint64_t)ORC_M) / n;
    f[s] = v < 1 ? 1 : (uint32_t)v;
    sum += f[s];
  }
  if (sum < (int64_t)ORC_M) {
    /* the whole deficit goes to the largest frequency (ties: smaller s) */
    int best = -1;
    for (int s = 0; s < 256; s++)
      if (f[s] && (best < 0 || f[s] > f[best])) best = s;
    f[best] += (uint32_t)(ORC_M - sum);
  }
  while (sum > (int64_t)ORC_M) {
    /* too many forced-to-one symbols: take one from the largest f > 1 */
    int best = -1;
    for (int s = 0; s < 256; s++)
      if (f[s] > 1 && (best < 0 || f[s] > f[best])) best = s;
    if (best < 0) return orc_fail(ORC_E_ARG, "normalize: cannot fit");
    f[best]--;
    sum--;
  }
  for (int s = 0; s < 256; s++) freq[s] = (uint16_t)f[s];
  return ORC_OK;
}

uint32_t orc_table_size(const uint16_t* freq) {
  uint32_t present = 0;
  for (int s = 0; s < 256; s++) present += freq[s] != 0;
  return (32 + 2 * present + 3) & ~3u;
}

void orc_table_write(const uint16_t* freq, uint8_t* out) {
  uint32_t sz = orc_table_size(freq);
  memset(out, 0, sz);
  uint8_t* q = out + 32;
  for (int s = 0; s < 256; s++) {
    if (!freq[s]) continue;
    out[s >> 3] |= (uint8_t)(1u << (s & 7));
    wr16(q, (uint16_t)(freq[s] - 1));
    q += 2;
  }
}

int orc_table_read(const uint8_t* p, uint32_t avail, uint16_t* freq) {
  if (avail < 32) return orc_fail(ORC_E_CORRUPT, "table: truncated bitmap");
  uint32_t present = 0, total = 0;
  for (int s = 0; s < 256; s++) present += (p[s >> 3] >> (s & 7)) & 1;
  uint32_t sz = (32 + 2 * present + 3) & ~3u;
  if (present == 0) return orc_fail(ORC_E_CORRUPT, "table: no symbol present");
  if (sz > avail) return orc_fail(ORC_E_CORRUPT, "table: truncated");
  const uint8_t* q = p + 32;
  for (int s = 0; s < 256; s++) {
    if ((p[s >> 3] >> (s & 7)) & 1) {
      freq[s] = (uint16_t)(rd16(q) + 1);
      q += 2;
      total += freq[s];
    } else {
      freq[s] = 0;
    }
  }
  if (total != ORC_M) return orc_fail(ORC_E_CORRUPT, "table: frequencies sum to %u, not 4096", total);
  return (int)sz;
}

static void cumulative(const uint16_t* freq, uint32_t* cum) {
  uint32_t c = 0;
  for (int s = 0; s < 256; s++) {
    cum[s] = c;
    c += freq[s];
  }
}

int orc_rans_encode(const uint8_t* sym, uint32_t n, uint32_t W,
                    const uint16_t* freq, uint8_t* out, uint32_t cap,
                    uint32_t* out_len) {
  if (W < 1 || W > 64) return orc_fail(ORC_E_ARG, "rans: W=%u outside 1..64", W);
  uint32_t cum[256];
  cumulative(freq, cum);
  uint32_t x[64];
  for (uint32_t j = 0; j < W; j++) x[j] = ORC_L;
  /* at most one word per symbol */
  uint16_t* words = (uint16_t*)malloc(sizeof(uint16_t) * (n ? n : 1));
  if (!words) return orc_fail(ORC_E_NOMEM, "rans: out of memory");
  uint32_t nw = 0;
  for (uint32_t k = n; k-- > 0;) {
    uint32_t j = k % W;
    uint32_t f = freq[sym[k]];
    if (f == 0) {
      free(words);
      return orc_fail(ORC_E_ARG, "rans: symbol %u has zero frequency", sym[k]);
    }
    uint64_t xmax = ((uint64_t)(ORC_L >> ORC_PROB_BITS) << 16) * f; /* 2^20 * f */
    if (x[j] >= xmax) {
      words[nw++] = (uint16_t)(x[j] & 0xFFFF);
      x[j] >>= 16;
    }
    x[j] = (x[j] / f) * ORC_M + (x[j] % f) + cum[sym[k]];
  }
  uint32_t need = 4 * W + 2 * nw;
  if (need > cap) {
    free(words);
    return orc_fail(ORC_E_NOSPACE, "rans: need %u bytes", need);
  }
  for (uint32_t j = 0; j < W; j++) wr32(out + 4 * j, x[j]);
  for (uint32_t i = 0; i < nw; i++) wr16(out + 4 * W + 2 * i, words[nw - 1 - i]);
  free(words);
  *out_len = need;
  return ORC_OK;
}

int orc_rans_decode(const uint8_t* data, uint32_t len, uint32_t n, uint32_t W,
                    const uint16_t* freq, uint8_t* sym_out) {
  if (W < 1 || W > 64) return orc_fail(ORC_E_ARG, "rans: W=%u outside 1..64", W);
  if (len < 4 * W || ((len - 4 * W) & 1))
    return orc_fail(ORC_E_CORRUPT, "rans: %u bytes cannot hold %u states and whole words", len, W);
  uint32_t cum[256];
  cumulative(freq, cum);
  /* slot -> symbol, written out from the cumulative frequencies */
  uint8_t slot_sym[ORC_M];
  for (int s = 0; s < 256; s++)
    for (uint32_t t = cum[s]; t < cum[s] + freq[s]; t++) slot_sym[t] = (uint8_t)s;
  uint32_t x[64];
  for (uint32_t j = 0; j < W; j++) {
    x[j] = rd32(data + 4 * j);
    if (x[j] < ORC_L) return orc_fail(ORC_E_CORRUPT, "rans: initial state %u below 2^16", j);
  }
  uint32_t nwords = (len - 4 * W) / 2, wpos = 0;
  const uint8_t* w = data + 4 * W;
  for (uint32_t i = 0; i < n; i++) {
    uint32_t j = i % W;
    uint32_t slot = x[j] & (ORC_M - 1);
    uint8_t s = slot_sym[slot];
    x[j] = freq[s] * (x[j] >> ORC_PROB_BITS) + slot - cum[s];
    if (x[j] < ORC_L) {
      if (wpos >= nwords) return orc_fail(ORC_E_CORRUPT, "rans: word stream over-run at symbol %u", i);
      x[j] = (x[j] << 16) | rd16(w + 2 * wpos);
      wpos++;
    }
    sym_out[i] = s;
  }
  for (uint32_t j = 0; j < W; j++)
    if (x[j] != ORC_L) return orc_fail(ORC_E_CORRUPT, "rans: final state of lane %u is %u, not 2^16", j, x[j]);
  if (wpos != nwords) return orc_fail(ORC_E_CORRUPT, "rans: %u of %u words unused", nwords - wpos, nwords);
  return ORC_OK;
}
