/*
 * oracle.h -- plain, slow, obviously-correct CPU reference of the two-layer
 * absolute-offset codec.  TEST INFRASTRUCTURE ONLY: only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code with the GPU library (paper_2606_24531_amd/csrc); the two
 * meet only at the archive byte format.
 *
 * What it follows:
 *  - Match layer: LZ77 whose back-references are absolute positions in the
 *    decompressed output, found by a global search, with the output cut into
 *    fixed-size blocks; since every match names an absolute position, a
 *    block can be decoded as soon as each earlier block its matches copy
 *    from is decoded (paper Section 2).
 *  - Entropy layer: per-block, per-stream rANS (Duda) interleaved over W
 *    states (Giesen), applied to each block on its own so that every block
 *    is an entry point (paper Sections 3 and 9).
 *  - Seek: decode of an absolute byte range through both layers (paper
 *    Section 5); its plain definition is decode_all(A)[lo:hi].
 *
 * All functions return 0 on success or a negative ORC_E_* code; the last
 * error text is available from orc_last_error().  Every buffer is owned by
 * the caller.
 */
#ifndef ACESEEK_ORACLE_H
#define ACESEEK_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0,
  ORC_E_ARG = -1,
  ORC_E_RANGE = -2,
  ORC_E_CORRUPT = -3,
  ORC_E_NOSPACE = -4,
  ORC_E_NOMEM = -7
};

/* Encoder parameters (encoder policy only: none of them changes decode). */
typedef struct {
  uint32_t block_size; /* B, bytes per block, 1 .. 2^24 */
  uint32_t interleave; /* W, rANS states per stream, 1 .. 64 */
  uint32_t min_match;  /* shortest match emitted, >= hash_len */
  uint32_t hash_len;   /* bytes hashed per position, 1 .. 64 */
  uint32_t max_chain;  /* candidates examined per position */
  uint32_t max_level;  /* 0 = unbounded; else every block level < max_level */
  uint32_t flags;      /* ORC_MODE_* stream-mode policy */
} orc_params;

/* Stream-mode policy (flags & 3). */
enum { ORC_MODE_AUTO = 0, ORC_MODE_RANS = 1, ORC_MODE_RAW = 2 };
/* flags bit 2: store offsets in 8 bytes even when every position fits in 4
 * (the format's width for outputs above 4 GiB; encoder policy only). */
enum { ORC_WIDE_OFFSETS = 4 };

const char* orc_last_error(void);
uint64_t orc_fnv1a64(const uint8_t* p, uint64_t n);

/* ---- entropy layer primitives (exposed for the closed-form pins) ---- */
/* Normalise symbol counts (256 entries, n = their sum > 0) to frequencies
 * summing to 4096, every present symbol >= 1. */
int orc_normalize(const uint64_t* counts, uint16_t* freq);
/* Encode n symbols with W interleaved states: writes W u32 states then the
 * u16 renormalisation words in decoder read order.  freq: 256 entries. */
int orc_rans_encode(const uint8_t* sym, uint32_t n, uint32_t W,
                    const uint16_t* freq, uint8_t* out, uint32_t cap,
                    uint32_t* out_len);
/* Decode n symbols from data produced by orc_rans_encode; checks that every
 * final state is 2^16 and that every word was consumed. */
int orc_rans_decode(const uint8_t* data, uint32_t len, uint32_t n, uint32_t W,
                    const uint16_t* freq, uint8_t* sym_out);

/* ---- archive ---- */
int orc_encode_bound(uint64_t n, const orc_params* p, uint64_t* bound);
int orc_encode(const uint8_t* src, uint64_t n, const orc_params* p,
               uint8_t* dst, uint64_t cap, uint64_t* out_len);
/* Assemble an archive from an explicit parse.  Tokens are listed block by
 * block: seq_count[b] sequences for block b, each (L, M, O).  The parse is
 * validated against x (it must reproduce x). */
int orc_assemble(const uint8_t* x, uint64_t n, uint32_t block_size,
                 uint32_t interleave, uint32_t flags, const uint32_t* seq_count,
                 const uint32_t* L, const uint32_t* M, const uint64_t* O,
                 uint8_t* dst, uint64_t cap, uint64_t* out_len);

/* Header facts. */
int orc_info(const uint8_t* a, uint64_t len, uint64_t* n_total,
             uint32_t* block_size, uint32_t* n_blocks, uint32_t* depth,
             uint32_t* interleave);
/* Full validation and sequential decode into out (cap >= n_total). */
int orc_decode(const uint8_t* a, uint64_t len, uint8_t* out, uint64_t cap);
/* The same decode with the blocks of each dependency level decoded in
 * parallel on `threads` host threads (0 = all; OpenMP), levels in order.
 * The all-cores CPU baseline; *threads_used receives the team size. */
int orc_decode_levels(const uint8_t* a, uint64_t len, uint8_t* out, uint64_t cap, int threads,
                      int* threads_used);
/* out[0 .. hi-lo) = decode(a)[lo:hi). */
int orc_seek(const uint8_t* a, uint64_t len, uint64_t lo, uint64_t hi,
             uint8_t* out);
/* Blocks needed to decode [lo,hi): the targets and, transitively, every block
 * holding a source byte.  Writes a 0/1 flag per block into need[n_blocks]
 * and the count into *count. */
int orc_closure(const uint8_t* a, uint64_t len, uint64_t lo, uint64_t hi,
                uint8_t* need, uint32_t* count);
/* Per-block facts read back from a validated archive (for tests):
 * level[b], n_seq[b], and for each stream s in {LIT, LEN, OFF} its mode. */
int orc_block_facts(const uint8_t* a, uint64_t len, uint32_t* level,
                    uint32_t* n_seq, uint8_t* modes /* 3 per block */);
/* The decoded token streams of one block (after the entropy layer):
 * lit (cap B), lens (u16 L, u16 M per sequence), offs (u64 per sequence). */
int orc_block_tokens(const uint8_t* a, uint64_t len, uint32_t block,
                     uint8_t* lit, uint32_t* n_lit, uint32_t* Ls, uint32_t* Ms,
                     uint64_t* Os, uint32_t* n_seq);

#ifdef __cplusplus
}
#endif
#endif
