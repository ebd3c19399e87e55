/* Internal helpers of the CPU oracle (test infrastructure only). */
#ifndef ACESEEK_ORACLE_INTERNAL_H
#define ACESEEK_ORACLE_INTERNAL_H
#include <stdint.h>
#include <stddef.h>
#include "oracle.h"

/* Archive layout constants (the byte format both sides read). */
#define ORC_MAGIC 0x314B5341u /* "ASK1" little-endian */
#define ORC_VERSION 1
#define ORC_HDR 64
#define ORC_BLK 32
#define ORC_SDESC 16
#define ORC_NSTREAM 3
#define ORC_STREAM_LIT 0
#define ORC_STREAM_LEN 1
#define ORC_STREAM_OFF 2
#define ORC_PROB_BITS 12
#define ORC_M 4096u
#define ORC_L 65536u

int orc_fail(int code, const char* fmt, ...);

static inline uint16_t rd16(const uint8_t* p) { return (uint16_t)(p[0] | (p[1] << 8)); }
static inline uint32_t rd32(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}
static inline uint64_t rd64(const uint8_t* p) { return (uint64_t)rd32(p) | ((uint64_t)rd32(p + 4) << 32); }
static inline void wr16(uint8_t* p, uint16_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); }
static inline void wr32(uint8_t* p, uint32_t v) {
  p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); p[2] = (uint8_t)(v >> 16); p[3] = (uint8_t)(v >> 24);
}
static inline void wr64(uint8_t* p, uint64_t v) { wr32(p, (uint32_t)v); wr32(p + 4, (uint32_t)(v >> 32)); }

/* Size of the serialised frequency table: 32-byte presence bitmap plus one
 * u16 per present symbol, padded to a multiple of 4. */
uint32_t orc_table_size(const uint16_t* freq);
void orc_table_write(const uint16_t* freq, uint8_t* out);
/* Parses a table; returns its size in bytes or a negative error. */
int orc_table_read(const uint8_t* p, uint32_t avail, uint16_t* freq);

#endif
