/* Error reporting and FNV-1a-64 for the CPU oracle (test infrastructure). */
#include <stdarg.h>
#include <stdio.h>
#include "internal.h"

static __thread char g_err[512];

int orc_fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

const char* orc_last_error(void) { return g_err; }

/* FNV-1a, 64-bit: offset basis 0xcbf29ce484222325, prime 0x100000001b3.
 * The paper checks decoded output by an FNV hash against the original
 * (Section 4); the byte comparison is the actual proof. */
uint64_t orc_fnv1a64(const uint8_t* p, uint64_t n) {
  uint64_t h = 0xcbf29ce484222325ull;
  for (uint64_t i = 0; i < n; i++) {
    h ^= p[i];
    h *= 0x100000001b3ull;
  }
  return h;
}
