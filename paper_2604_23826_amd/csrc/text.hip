// Text ingest fused with the reduction (p <= 16).
//
// The data start as CSV text (section "Validation and Infrastructure
// Testing"; section "Data Representation and Sufficient Statistics" on the
// cost of repeated parsing).  Here a chunk of text in HBM is parsed once, on
// the GPU, and every parsed row goes straight into the same shifted column
// sums and X^T X accumulators as the binary path; nothing is written back.
//
// Work split: workgroup w owns the lines whose first byte lies in
// [w seg, (w + 1) seg), seg a multiple of 4096 up to 40 KiB chosen per chunk
// from its mean line length (pick_text_seg); its threads find the line starts
// of seg / 256-byte slices, then take the lines in turn, one per thread and
// round.  The workgroup stages its bytes (plus MAXLINE bytes of the next
// segment, for lines that run past the end) in LDS with 16 bytes of padding
// per 256, so that threads reading their own slices hit different banks.  The
// block shift is the workgroup's first line.
//
// Fields: integer columns are decimal integers (optional sign, at most 18
// digits), parsed exactly; other columns are decimal numbers (optional sign,
// digits with an optional point, optional exponent), converted to the nearest
// FP64 value: the decimal significand w and exponent q give w * 10^q, formed
// as an exact 256-bit integer ratio and divided once with correct rounding.
// The ratio's range: every |value| below 1e73 whose last written digit has
// exponent q >= -57 converts; a field beyond 2^247 (about 2.3e74) or with
// q < -57 is refused as malformed (in between, by the significand's bit
// length).  A malformed field marks
// the handle (STATS_E_PARSE, smallest byte offset) and its row is skipped.
#include <cmath>
#include <cstring>

#include "accum_common.hpp"
#include "runtime.hpp"

namespace st {
namespace text {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int SEG = 1 << 15;     // bytes of line starts per workgroup (conversion, line counts)
constexpr int SEG_MAX = 40 << 10;  // the fused kernel's segments: a multiple of 4096 up to this (chosen per chunk)
constexpr int MAXLINE = 4096;    // longest line accepted
constexpr int SLICE = SEG / 256;  // bytes of line starts per thread (one slice per thread)
constexpr int SLICE_MAX = SEG_MAX / 256;
constexpr int MAXLS = 2048;      // line starts per workgroup kept in the table
constexpr int STAGE = 32 + SEG_MAX + MAXLINE;  // + up to 15 bytes of alignment in front
constexpr int STAGE_PADDED = STAGE + (STAGE / 256 + 2) * 16;  // room for word reads past the end

struct Args {
  const char* buf;
  int64_t nbytes;  // readable bytes
  int64_t nend;    // lines start before nend; the last one may end at nend
  int p;
  uint32_t intmask;
  int64_t base_off;  // offset of buf in the caller's stream (for messages)
  int seg;           // bytes of line starts per workgroup: a multiple of 4096, at most SEG_MAX
  acc::Args acc;
  DevStatus* status;
};

__device__ inline int pad(int i) { return i + ((i >> 8) << 4); }


// Staged text [w0, w0 + n) of the chunk.  The parser works on positions
// relative to w0 (32-bit); positions at or past lim (min(nend, w0 + n) - w0)
// read as -1.
struct Stage {
  const unsigned char* s;
  int64_t w0;  // stream offset of staged byte 0
  int n;       // staged bytes
  int lim;     // first relative position that is not text of this chunk
};

// A thread's reader of the staged text (one LDS byte per character; the
// staged bytes are padded 16 per 256 so that threads reading their own slices
// fall on different banks).
struct Cur {
  const Stage* S;
  __device__ explicit Cur(const Stage& st) : S(&st) {}
  __device__ inline int at(int pos) const {
    if (pos >= S->lim) return -1;
    return ((const __attribute__((address_space(3))) unsigned char*)S->s)[pad(pos)];
  }
  // The four bytes at pos .. pos + 3 (the first in the low byte), from two
  // aligned LDS words; bytes at or past lim read as 0xFF.  pos >= 0.
  __device__ inline uint32_t word4(int pos) const {
    const int a = pos & ~3;
    const __attribute__((address_space(3))) unsigned char* b =
        (const __attribute__((address_space(3))) unsigned char*)S->s;
    const uint32_t lo = *(const __attribute__((address_space(3))) uint32_t*)(b + pad(a));
    const uint32_t hi = *(const __attribute__((address_space(3))) uint32_t*)(b + pad(a + 4));
    uint32_t v = __builtin_amdgcn_alignbyte(hi, lo, (uint32_t)(pos & 3));
    const int room = S->lim - pos;
    if (room < 4) v |= room <= 0 ? 0xFFFFFFFFu : (0xFFFFFFFFu << (8 * room));
    return v;
  }
};

// Leading decimal digits of a 4-byte word (first character in the low byte):
// their count k (0..4) and value.  A byte is a digit when its high nibble is
// 3 and its low nibble is below 10 (low nibble + 6 does not carry into bit 4).
__device__ inline int digit_run(uint32_t v, uint32_t* val) {
  const uint32_t m = ((v & 0xF0F0F0F0u) ^ 0x30303030u) | (((v & 0x0F0F0F0Fu) + 0x06060606u) & 0xF0F0F0F0u);
  const int k = m ? (__builtin_ctz(m) >> 3) : 4;
  // digit values moved to the top k bytes (leading zero bytes add nothing);
  // then bytes (b0 b1 b2 b3) -> (10 b0 + b1, 10 b2 + b3) -> 100 (..) + (..)
  const uint32_t y = k ? (v & 0x0F0F0F0Fu) << (8 * (4 - k)) : 0u;
  const uint32_t t = y * 10u + (y >> 8);
  *val = (t & 0xFFu) * 100u + ((t >> 16) & 0xFFu);
  return k;
}

// Decimal digits of v < 10^4 without leading zeros.
__device__ inline int sig_count(uint32_t v) {
  return (v >= 1000u) + (v >= 100u) + (v >= 10u) + (v >= 1u);
}

__device__ inline uint32_t pow10_small(int k) {  // 10^k, 1 <= k <= 4
  return k >= 3 ? (k == 4 ? 10000u : 1000u) : (k == 2 ? 100u : 10u);
}

__device__ inline int bitlen64(uint64_t v) { return v ? 64 - __builtin_clzll(v) : 0; }
__device__ inline int bitlen128(u128 v) {
  const uint64_t hi = (uint64_t)(v >> 64);
  return hi ? 128 - __builtin_clzll(hi) : bitlen64((uint64_t)v);
}

__device__ inline U256 u256_mul_small(U256 a, uint32_t m) {
  U256 r;
  u128 carry = 0;
  for (int k = 0; k < 4; ++k) {
    const u128 t = (u128)a.w[k] * m + carry;
    r.w[k] = (uint64_t)t;
    carry = t >> 64;
  }
  return r;
}

// Correctly rounded value of (w + sticky) * 2^e2 where w has 54..128 bits
// and sticky marks a nonzero remainder below the last bit of w.
__device__ inline double round_to_double(u128 w, bool sticky, int e2, bool neg) {
  const int bl = bitlen128(w);
  const int extra = bl - 53;
  uint64_t m;
  if (extra > 0) {
    const u128 low = w & (((u128)1 << extra) - 1);
    const u128 half = (u128)1 << (extra - 1);
    m = (uint64_t)(w >> extra);
    if (low > half || (low == half && (sticky || (m & 1)))) ++m;
    e2 += extra;
  } else {
    m = (uint64_t)w << (-extra);
    e2 += extra;
  }
  if (m == ((uint64_t)1 << 53)) {
    m >>= 1;
    ++e2;
  }
  const double r = ldexp((double)m, e2);
  return neg ? -r : r;
}

struct Pow5 {
  uint64_t v[28];  // 5^k, k <= 27 (5^27 < 2^63)
};
constexpr Pow5 make_pow5() {
  Pow5 t{};
  uint64_t r = 1;
  for (int k = 0; k < 28; ++k) {
    t.v[k] = r;
    r *= 5;
  }
  return t;
}
__constant__ Pow5 kPow5 = make_pow5();

__device__ inline uint64_t pow5_u64(int k) { return kPow5.v[k]; }

// Exact w * 10^q for w < 2^64 and |q| <= 27: w 5^q fits 128 bits for q > 0;
// for q < 0 the quotient w 2^k / 5^-q (k chosen for 54..56 bits) comes from
// an FP64 estimate corrected with the exact 128-bit remainder.
__device__ inline double fast_decimal(uint64_t w, int q, bool neg) {
  if (q >= 0) return round_to_double((u128)w * pow5_u64(q), false, q, neg);
  const uint64_t D = pow5_u64(-q);
  const int bw = bitlen64(w), bd = bitlen64(D);
  const int k = 55 - bw + bd;  // w 2^k has 55 + bd <= 119 bits
  const u128 N = (u128)w << k;
  const double est = (double)N / (double)D;
  uint64_t Q = (uint64_t)est;  // within a few units of floor(N / D)
  __int128 rem = (__int128)N - (__int128)((u128)Q * D);
  while (rem < 0) {
    --Q;
    rem += D;
  }
  while (rem >= (__int128)D) {
    ++Q;
    rem -= D;
  }
  return round_to_double((u128)Q, rem != 0, -k + q, neg);
}

// Exact ratio path for everything else (more than 19 digits, |q| up to 57).
__device__ __attribute__((noinline)) double slow_decimal(u128 w, int q, bool sticky, bool neg) {
  U256 num = u256_from_u128(w), den = u256_from_u128((u128)1);
  if (sticky) {
    num = u256_mul_small(num, 10u);
    num.w[0] |= 1u;  // (10 w + 1) 10^(q - 1); the low digit was 0
    --q;
  }
  if (q >= 0)
    for (int k = 0; k < q; ++k) num = u256_mul_small(num, 10u);
  else
    for (int k = 0; k < -q; ++k) den = u256_mul_small(den, 10u);
  return u256_div_to_double(neg, num, den);
}

// Parses one field starting at f; on success returns the position of the
// terminating byte (',' or '\n' or nend) and the value bits in *bits (int64
// for integer columns, FP64 otherwise).  Returns -1 - pos on malformed input.
// Decimal text keeps 38 significant digits exactly plus a sticky digit for
// any further nonzero digit, which rounds like the full expansion whenever no
// FP64 rounding midpoint lies within 1e-38 relative (always, e.g., for
// printed doubles).  Significands of up to 19 digits (every integer field and
// printed double) are gathered in 64 bits; longer ones go through
// parse_wide.
struct Parsed {
  int pos;        // terminating byte, or -1 - pos on malformed input
  uint64_t bits;  // value
};
__device__ __attribute__((noinline)) Parsed parse_wide(Stage S, int f, bool is_int);

__device__ inline double decimal_value(u128 w, int nd, int q, bool sticky, bool neg, bool* bad) {
  if (w == 0) return neg ? -0.0 : 0.0;
  if (!sticky && nd <= 19 && q >= -27 && q <= 27) return fast_decimal((uint64_t)w, q, neg);
  // range of the exact ratio: 256-bit numerator and denominator
  const int lw = bitlen128(w);
  const int qq = sticky ? q - 1 : q;
  if (qq > 0 && lw + 4 + (qq * 3402 + 1023) / 1024 > 250) *bad = true;  // log2(10) < 3402/1024
  if (qq < -57) *bad = true;
  if (*bad) return 0.0;
  return slow_decimal(w, q, sticky, neg);
}

// Digits from position i on, four per step, into w (significant digits
// counted in nd; q lowered by one per digit when frac).  Returns the character
// after the digits (-1 past the text), or kTooLong when the run would give w
// more than 19 significant digits (w, nd, i are then unspecified).
constexpr int kTooLong = -2;
__device__ inline int digit_steps(const Cur& C, int& i, uint64_t& w, int& nd, int& q, bool frac) {
  for (;;) {
    const uint32_t v = C.word4(i);
    uint32_t val;
    const int k = digit_run(v, &val);
    if (k) {
      const int sig = w ? k : sig_count(val);
      if (nd + sig > 19) return kTooLong;
      w = w * pow10_small(k) + val;
      nd += sig;
      i += k;
      if (frac) q -= k;
    }
    if (k < 4) return i >= C.S->lim ? -1 : (int)((v >> (8 * k)) & 0xFFu);
  }
}

__device__ inline int parse_field(Cur& C, int f, bool is_int, uint64_t* bits) {
  int i = f;
  int c = C.at(i);
  bool neg = false;
  if (c == '-' || c == '+') {
    neg = c == '-';
    ++i;
  }
  uint64_t w = 0;
  int nd = 0;
  int q = 0;
  const int i0 = i;
  c = digit_steps(C, i, w, nd, q, false);
  if (c == kTooLong) {
    const Parsed r = parse_wide(*C.S, f, is_int);
    *bits = r.bits;
    return r.pos;
  }
  bool digits = i > i0;
  if (is_int) {
    if (!digits || nd > 18) return -1 - i;
    if (c != ',' && c != '\n' && c != -1) return -1 - i;
    const int64_t v = (int64_t)w;
    *bits = (uint64_t)(neg ? -v : v);
    return i;
  }
  if (c == '.') {
    ++i;
    const int i1 = i;
    c = digit_steps(C, i, w, nd, q, true);
    if (c == kTooLong) {
      const Parsed r = parse_wide(*C.S, f, is_int);
      *bits = r.bits;
      return r.pos;
    }
    digits |= i > i1;
  }
  if (!digits) return -1 - i;
  if (c == 'e' || c == 'E') {
    c = C.at(++i);
    bool eneg = false;
    if (c == '-' || c == '+') {
      eneg = c == '-';
      c = C.at(++i);
    }
    int ex = 0;
    bool ed = false;
    while (c >= '0' && c <= '9') {
      ed = true;
      if (ex < 100000) ex = ex * 10 + (c - '0');
      c = C.at(++i);
    }
    if (!ed) return -1 - i;
    q += eneg ? -ex : ex;
  }
  if (c != ',' && c != '\n' && c != -1) return -1 - i;
  bool bad = false;
  const double v = decimal_value((u128)w, nd, q, false, neg, &bad);
  if (bad) return -1 - f;
  *bits = (uint64_t)__double_as_longlong(v);
  return i;
}

// The same for significands of more than 19 digits: 128-bit accumulation.
__device__ __attribute__((noinline)) Parsed parse_wide(Stage S, int f, bool is_int) {
  Cur C(S);
  Parsed out{0, 0};
  int i = f;
  int c = C.at(i);
  bool neg = false;
  if (c == '-' || c == '+') {
    neg = c == '-';
    c = C.at(++i);
  }
  u128 w = 0;
  int nd = 0;
  int q = 0;
  bool digits = false, sticky = false;
  while (c >= '0' && c <= '9') {
    digits = true;
    const int d = c - '0';
    if (w != 0 || d != 0) {
      if (nd < 38) {
        w = w * 10 + (u128)d;
        ++nd;
      } else {
        sticky |= d != 0;
        ++q;
      }
    }
    c = C.at(++i);
  }
  if (is_int) return Parsed{-1 - i, 0};  // more than 18 digits
  if (c == '.') {
    c = C.at(++i);
    while (c >= '0' && c <= '9') {
      digits = true;
      const int d = c - '0';
      if (w == 0 && d == 0) {
        --q;
      } else if (nd < 38) {
        w = w * 10 + (u128)d;
        ++nd;
        --q;
      } else {
        sticky |= d != 0;
      }
      c = C.at(++i);
    }
  }
  if (!digits) return Parsed{-1 - i, 0};
  if (c == 'e' || c == 'E') {
    c = C.at(++i);
    bool eneg = false;
    if (c == '-' || c == '+') {
      eneg = c == '-';
      c = C.at(++i);
    }
    int ex = 0;
    bool ed = false;
    while (c >= '0' && c <= '9') {
      ed = true;
      if (ex < 100000) ex = ex * 10 + (c - '0');
      c = C.at(++i);
    }
    if (!ed) return Parsed{-1 - i, 0};
    q += eneg ? -ex : ex;
  }
  if (c != ',' && c != '\n' && c != -1) return Parsed{-1 - i, 0};
  bool bad = false;
  const double v = decimal_value(w, nd, q, sticky, neg, &bad);
  if (bad) return Parsed{-1 - f, 0};
  out.pos = i;
  out.bits = (uint64_t)__double_as_longlong(v);
  return out;
}

// ---- fast path for the common field forms -----------------------------------
//
// Bytes [pos, pos + 20) of the staged text in five words (first character in
// the low byte of w[0]); positions at or past lim read as 0xFF.  pos <= lim,
// so every word read lies inside the staging buffer.
__device__ inline void window20(const Cur& C, int pos, uint32_t (&w)[5]) {
  const __attribute__((address_space(3))) unsigned char* b =
      (const __attribute__((address_space(3))) unsigned char*)C.S->s;
  const int a = pos & ~3;
  uint32_t r[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) r[j] = *(const __attribute__((address_space(3))) uint32_t*)(b + pad(a + 4 * j));
  const uint32_t sh = (uint32_t)(pos & 3);
#pragma unroll
  for (int j = 0; j < 5; ++j) w[j] = __builtin_amdgcn_alignbyte(r[j + 1], r[j], sh);
  const int room = C.S->lim - pos;
  if (room < 20) {
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const int rj = room - 4 * j;
      w[j] |= rj <= 0 ? 0xFFFFFFFFu : (rj < 4 ? (0xFFFFFFFFu << (8 * rj)) : 0u);
    }
  }
}

__device__ inline uint32_t pow10_upto4(int k) {  // 10^k, 0 <= k <= 4, without branches
  return k == 4 ? 10000u : (uint32_t)(0x03E80064000A0001ull >> (16 * k)) & 0xFFFFu;
}

// The leading decimal digits of the 4 NW bytes w[0..NW-1]: their count k
// (0..4 NW), appended to *val (*val = *val 10^k + their value; wraps modulo
// 2^64, which only matters past 19 digits), and the byte after them in *term
// (0xFF when all 4 NW bytes are digits).  Four digits per step (the SWAR step
// of digit_run); the steps stop when no lane of the wave has digits left.
template <int NW>
__device__ inline int lead_digits(const uint32_t (&w)[5], uint64_t* val, uint32_t* term) {
  uint64_t v = *val;
  int k = 0;
  bool done = false;
  uint32_t t8 = 0xFFu;
#pragma unroll
  for (int j = 0; j < NW; ++j) {
    if (j > 0 && __builtin_amdgcn_ballot_w64(!done) == 0) break;  // wave-uniform
    const uint32_t x = w[j];
    const uint32_t m = ((x & 0xF0F0F0F0u) ^ 0x30303030u) | (((x & 0x0F0F0F0Fu) + 0x06060606u) & 0xF0F0F0F0u);
    const int kw = m ? (__builtin_ctz(m) >> 3) : 4;
    const int kj = done ? 0 : kw;
    const uint32_t y = kj ? (x & 0x0F0F0F0Fu) << (8 * (4 - kj)) : 0u;
    const uint32_t t = y * 10u + (y >> 8);
    v = v * pow10_upto4(kj) + ((t & 0xFFu) * 100u + ((t >> 16) & 0xFFu));
    if (!done && kw < 4) t8 = (x >> (8 * kw)) & 0xFFu;
    k += kj;
    done |= kw < 4;
  }
  *val = v;
  *term = t8;
  return k;
}

// The field at f when it has one of the common forms: [sign] 1..15 digits
// (integer columns), or [sign] digits [. digits] with 1..19 digits in all and
// no exponent (decimal columns).  Then it returns true with the terminator's
// position in *end, its byte in *term (-1 past the text) and the value bits in
// *bits, exactly as parse_field gives them (the same w, digit count and q go
// to decimal_value); otherwise false, and parse_field takes the field.
__device__ inline bool fast_field(const Cur& C, int f, bool is_int, int* end, int* term, uint64_t* bits) {
  uint32_t w[5];
  window20(C, f, w);
  const uint32_t c0 = w[0] & 0xFFu;
  const bool neg = c0 == '-';
  const uint32_t sg = (c0 == '-' || c0 == '+') ? 1u : 0u;
#pragma unroll
  for (int j = 0; j < 4; ++j) w[j] = __builtin_amdgcn_alignbyte(w[j + 1], w[j], sg);
  uint64_t v = 0;
  uint32_t t1;
  const int k1 = lead_digits<4>(w, &v, &t1);
  if (k1 > 15) return false;
  int p = f + (int)sg + k1;  // the byte after the digits
  int c = p >= C.S->lim ? -1 : (int)t1;
  int nd = k1, q = 0;
  if (!is_int && c == '.') {
    // fraction digits appended to v: w = (integer digits)(fraction digits)
    int k2 = 0;
    ++p;
    if (p < C.S->lim) {
      uint32_t w2[5], t2;
      window20(C, p, w2);
      k2 = lead_digits<5>(w2, &v, &t2);
      if (k1 + k2 > 19) return false;
      c = p + k2 >= C.S->lim ? -1 : (int)t2;
    } else {
      c = -1;
    }
    nd = k1 + k2;
    q = -k2;
    p += k2;
  }
  if (nd == 0 || (c != ',' && c != '\n' && c != -1)) return false;
  if (is_int) {
    const int64_t x = (int64_t)v;
    *bits = (uint64_t)(neg ? -x : x);
  } else {
    bool bad = false;
    const double d = decimal_value((u128)v, nd, q, false, neg, &bad);
    if (bad) return false;
    *bits = (uint64_t)__double_as_longlong(d);
  }
  *end = p;
  *term = c;
  return true;
}

// parse_field out of line, for the fields fast_field does not take.
__device__ __attribute__((noinline)) Parsed slow_field(Stage S, int f, bool is_int) {
  Cur C(S);
  uint64_t bits = 0;
  const int r = parse_field(C, f, is_int, &bits);
  return Parsed{r, bits};
}

// Parses the line starting at L (P fields) into row[0..P), each field through
// fast_field first, else parse_field.  Returns the position of its end ('\n'
// or nend), or -1 - end on a malformed line (*bad_at = the offending field's
// offset).
template <int P>
__device__ inline int parse_line_p(const Args& a, Cur& C, int L, uint64_t (&row)[P], int* bad_at) {
  int f = L;
#pragma unroll
  for (int c = 0; c < P; ++c) {
    const bool is_int = (a.intmask >> c) & 1u;
    uint64_t bits = 0;
    int r, term;
    if (!fast_field(C, f, is_int, &r, &term, &bits)) {
      const Parsed sp = slow_field(*C.S, f, is_int);
      r = sp.pos;
      bits = sp.bits;
      term = r >= 0 ? C.at(r) : 0;
    }
    const bool last = c == P - 1;
    const bool ok = r >= 0 && (last ? (term == '\n' || term == -1) : term == ',');
    if (!ok) {
      *bad_at = f;
      int e = r >= 0 ? r : -1 - r;  // skip to the end of the line
      for (;;) {
        const int ch = C.at(e);
        if (ch == '\n' || ch < 0) break;
        ++e;
      }
      return -1 - e;
    }
    row[c] = bits;
    if (last) return r;
    f = r + 1;
  }
  return f;
}

// Copies the text [w0r, w0r + nr) of buf into LDS (padded 16 bytes per 256)
// on a 16-byte aligned origin: LDS position i holds stream byte w0r - sh + i,
// sh = the misalignment of buf + w0r, which is returned.  Every thread issues
// its aligned 16-byte loads before its first LDS write; the vectors at the
// two ends are assembled byte by byte so that nothing outside
// [buf + w0r - (w0r >= 16 ? sh : 0), buf + w0r + nr) is read (positions before
// w0r hold zeros when w0r < 16, earlier stream bytes otherwise).
__device__ inline int stage_text(const char* buf, int64_t w0r, int nr, unsigned char* s_buf) {
  const int sh = (int)((uintptr_t)(buf + w0r) & 15u);
  const char* base = buf + w0r - sh;
  const int tot = sh + nr;
  const int nv = (tot + 15) >> 4;
  constexpr int NVT = (STAGE + 15) / 16 / kThreads + 1;
  u32x4 q[NVT];
#pragma unroll
  for (int u = 0; u < NVT; ++u) {
    const int v = (int)threadIdx.x + u * kThreads;
    q[u] = (u32x4){0u, 0u, 0u, 0u};
    if (v < nv) {
      const int p0 = 16 * v;
      if (p0 + 16 <= tot && (w0r >= 16 || p0 >= sh)) {
        q[u] = *(const u32x4*)(base + p0);
      } else {
        uint32_t wd[4] = {0u, 0u, 0u, 0u};
        for (int k = 0; k < 16; ++k) {
          const int pos = p0 + k;
          if (pos >= sh && pos < tot)
            wd[k >> 2] |= (uint32_t)(unsigned char)buf[w0r + pos - sh] << (8 * (k & 3));
        }
        q[u] = (u32x4){wd[0], wd[1], wd[2], wd[3]};
      }
    }
  }
#pragma unroll
  for (int u = 0; u < NVT; ++u) {
    const int v = (int)threadIdx.x + u * kThreads;
    if (v < nv) *(__attribute__((address_space(3))) u32x4*)(s_buf + pad(16 * v)) = q[u];
  }
  return sh;
}

// Line starts of a workgroup's segment [s0r, s1r) (stage-relative; a line
// starts after '\n' or at the stream start).  Thread t finds the newlines of
// its slice (slice positions, a multiple of 16 up to SLICE_MAX) in one pass
// of 16-byte LDS reads, keeping them as a bit
// mask (a '\n' byte is a zero byte of v ^ 0x0a0a0a0a); a workgroup scan of the
// counts places them in s_ls in stream order when they fit (<= MAXLS).
// Returns their number; *c0, *c1 receive this thread's slice and *before the
// number of line starts in earlier slices (the index of its first line).
// Contains barriers: every thread of the workgroup calls it.
__device__ inline int line_starts(const unsigned char* s_buf, int64_t w0, int s0r, int s1r, int slice,
                                  unsigned short* s_ls, int* s_wsum, int* c0_out, int* c1_out,
                                  int* before_out) {
  static_assert(SLICE * kThreads == SEG && SLICE % 16 == 0 && SLICE_MAX % 16 == 0, "one slice per thread");
  constexpr int NV = SLICE_MAX / 16 + 1;     // 16-byte reads per slice (it may start mid-vector)
  constexpr int NM = (16 * NV + 31) / 32;    // 32-bit mask words
  const int c0 = s0r + (int)threadIdx.x * slice;
  const int c1 = min(c0 + slice, s1r);
  // newline positions m in [mlo, mhi) start the lines c0 .. c1 - 1; bit b of the
  // mask is position mb + b
  const int mlo = max(c0 - 1, 0), mhi = c1 - 1;
  const int mb = mlo & ~15;
  uint32_t nl[NM];
#pragma unroll
  for (int j = 0; j < NM; ++j) nl[j] = 0;
  int mine = 0;
  if (c0 < c1) {
    if (w0 + c0 == 0) ++mine;  // the stream's first byte
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int m16 = mb + 16 * k;
      if (m16 < mhi) {
        const u32x4 v = *(const __attribute__((address_space(3))) u32x4*)(
            (const __attribute__((address_space(3))) unsigned char*)s_buf + pad(m16));
        uint32_t bits = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const uint32_t x = v[e] ^ 0x0A0A0A0Au;
          const uint32_t z = ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x | 0x7F7F7F7Fu);  // 0x80 per '\n'
          // bits 7, 15, 23, 31 -> bits 0..3 (the four shifted copies do not overlap)
          bits |= (((z >> 7) * 0x204081u) >> 21 & 0xFu) << (4 * e);
        }
        // keep positions in [mlo, mhi)
        const int b0 = mlo - m16, b1 = mhi - m16;
        if (b0 > 0) bits &= 0xFFFFu << b0;
        if (b1 < 16) bits &= (1u << b1) - 1u;
        nl[k >> 1] |= bits << (16 * (k & 1));
      }
    }
#pragma unroll
    for (int j = 0; j < NM; ++j) mine += __builtin_popcount(nl[j]);
  }
  // workgroup exclusive scan of the counts
  int incl = mine;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) s_wsum[wv] = incl;
  __syncthreads();
  int before = incl - mine, total = 0;
  for (int k = 0; k < kThreads / 64; ++k) {
    if (k < wv) before += s_wsum[k];
    total += s_wsum[k];
  }
  if (total <= MAXLS && c0 < c1) {
    int at = before;
    if (w0 + c0 == 0) s_ls[at++] = (unsigned short)c0;
#pragma unroll
    for (int j = 0; j < NM; ++j) {
      uint32_t m = nl[j];
      while (m) {
        s_ls[at++] = (unsigned short)(mb + 32 * j + __builtin_ctz(m) + 1);
        m &= m - 1;
      }
    }
  }
  __syncthreads();
  *c0_out = c0;
  *c1_out = c1;
  *before_out = before;
  return total;
}

typedef double d4 __attribute__((ext_vector_type(4)));

// Waits for this wave's LDS accesses; also keeps the compiler from moving
// LDS accesses across it (the rows a wave stages are read by other lanes).
__device__ inline void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Products on the FP64 matrix cores: each wave stages the shifted rows of its
// lanes' lines, 32 at a time, in its own LDS rows; for v_mfma_f64_16x16x4f64
// a lane then holds column (lane % 16) of staged row 4 m + lane / 16, at once
// its element of the A operand (column i, row k) and of the B operand (row k,
// column j), so 8 products give the 32 rows' upper triangle; absent or
// malformed lines stage zeros.  The column sums are kept per lane.  For
// integer columns every partial sum is an integer below 2^53 under the guard
// checked by the merge, so the matrix-core sums are exact; the order of all
// sums is fixed, so results are bitwise reproducible.
template <int P>
__global__ __launch_bounds__(kThreads, 2) void k_text(Args a) {
  constexpr int T = P * (P + 1) / 2;
  constexpr int NWV = kThreads / 64;
  __shared__ __attribute__((aligned(16))) unsigned char s_buf[STAGE_PADDED];
  __shared__ uint64_t s_rows[NWV][32 * P];  // per wave: 32 staged rows (raw field bits)
  __shared__ int s_valid[NWV][32];
  __shared__ uint64_t sKb[P];
  __shared__ unsigned long long s_n;
  __shared__ unsigned short s_ls[MAXLS];  // line starts (stage-relative)
  __shared__ int s_wsum[NWV];
  static_assert(STAGE_PADDED >= NWV * 5 * 64 * 8, "the final reduction reuses the text stage");
  const int64_t s0 = (int64_t)blockIdx.x * a.seg;
  const int64_t s1 = min(s0 + (int64_t)a.seg, a.nend);
  const int64_t w0r = s0 >= 16 ? s0 - 16 : 0;  // first stream byte staged
  const int64_t w1 = min(s1 + (int64_t)MAXLINE, a.nbytes);
  // w0: stream offset of LDS position 0 (the staging origin is aligned)
  const int64_t w0 = w0r - stage_text(a.buf, w0r, (int)(w1 - w0r), s_buf);
  const int n = (int)(w1 - w0);
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();
  const Stage S{s_buf, w0, n, (int)(min(a.nend, w0 + (int64_t)n) - w0)};
  const int s0r = (int)(s0 - w0), s1r = (int)(s1 - w0);  // relative positions
  Cur C(S);

  int c0, c1, before;
  const int total = line_starts(s_buf, w0, s0r, s1r, a.seg / kThreads, s_ls, s_wsum, &c0, &c1, &before);
  (void)before;
  const bool table = total <= MAXLS;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, rsub = lane >> 4;
  uint64_t* wr = s_rows[wave];
  int* wv = s_valid[wave];
  d4 acc = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};  // even and odd steps
  double colsum = 0.0;
  unsigned long long nrows = 0;
  int first_bad = INT32_MAX;
  // this lane's column of the products and its shift
  const bool colv = col < P;
  const bool colint = colv && ((a.intmask >> col) & 1u);
  double Kc = 0.0;
  int64_t Kic = 0;
  // this lane's lines: table entries threadIdx.x, + 256, ...; or, when the
  // table overflowed, the lines starting in its own slice
  int idx = threadIdx.x;
  int Lc = c0;
  if (!table && w0 + Lc > 0)
    while (Lc < c1 && C.at(Lc - 1) != '\n') ++Lc;
  for (int round = 0;; ++round) {
    bool have;
    int L;
    if (table) {
      have = idx < total;
      L = have ? (int)s_ls[idx] : 0;
      idx += kThreads;
    } else {
      have = Lc < c1;
      L = Lc;
    }
    // every wave runs round 0 (its barrier); later rounds while a lane has a line
    if (round > 0 && __builtin_amdgcn_ballot_w64(have) == 0) break;
    uint64_t row[P];
    bool ok = false;
    if (have) {
      int bad_at = INT32_MAX;
      const int end = parse_line_p<P>(a, C, L, row, &bad_at);
      ok = end >= 0;
      if (ok) {
        ++nrows;
        Lc = end + 1;
      } else {
        first_bad = min(first_bad, bad_at);
        Lc = (-1 - end) + 1;
      }
    }
    if (round == 0) {
      // block shift: the row of thread 0's first line (the workgroup's first
      // line when the table holds them all), zeros if it does not parse
      if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < P; ++c) sKb[c] = ok ? row[c] : 0;
      }
      __syncthreads();
      const uint64_t kb = colv ? sKb[col] : 0;
      Kic = colint ? (int64_t)kb : 0;
      Kc = colint ? (double)Kic : __longlong_as_double((long long)kb);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if ((lane >> 5) == h) {
        if (ok) {
#pragma unroll
          for (int c = 0; c < P; ++c) wr[(lane & 31) * P + c] = row[c];
        }
        wv[lane & 31] = ok;
      }
      wave_lds_sync();
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int sr = 4 * m + rsub;
        double v = 0.0;
        if (colv && wv[sr]) {
          const uint64_t b = wr[sr * P + col];
          v = colint ? (double)((int64_t)b - Kic) : __longlong_as_double((long long)b) - Kc;
        }
        colsum += v;
        if (m & 1) acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(v, v, acc2, 0, 0, 0);
        else acc = __builtin_amdgcn_mfma_f64_16x16x4f64(v, v, acc, 0, 0, 0);
      }
      wave_lds_sync();
    }
  }
  if (first_bad != INT32_MAX) {
    atomicMin(&a.status->parse_off, (unsigned long long)(a.base_off + w0 + first_bad));
    atomicOr(&a.status->bits, ST_PARSE);
  }
  atomicAdd(&s_n, nrows);
  __syncthreads();  // the text stage is free: it holds the per-wave sums now
  double* red = (double*)s_buf;  // [wave][4 registers + 1 sum][64 lanes]
#pragma unroll
  for (int r = 0; r < 4; ++r) red[(wave * 5 + r) * 64 + lane] = acc[r] + acc2[r];
  red[(wave * 5 + 4) * 64 + lane] = colsum;
  __syncthreads();
  const acc::Args& ra = a.acc;
  uint64_t* out = ra.rec + (int64_t)blockIdx.x * (2 + 2 * P + T);
  for (int e = threadIdx.x; e < 4 * 64; e += kThreads) {
    // register r of lane l holds D[4r + l/16][l%16]
    const int r = e >> 6, l = e & 63;
    const int i = 4 * r + (l >> 4), j = l & 15;
    if (i <= j && j < P) {
      double v = red[r * 64 + l];
#pragma unroll
      for (int w = 1; w < NWV; ++w) v += red[(w * 5 + r) * 64 + l];
      const int t = i * P - i * (i - 1) / 2 + (j - i);
      out[2 + P + ra.dst[P + t]] = (uint64_t)__double_as_longlong(v);
    }
  }
  if (threadIdx.x < P) {
    const int c = threadIdx.x;
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < NWV; ++w)
#pragma unroll
      for (int k = 0; k < 4; ++k) v += red[(w * 5 + 4) * 64 + c + 16 * k];
    out[2 + P + ra.dst[c]] = (uint64_t)__double_as_longlong(v);
    // the shift word: the int64 value for integer columns, FP64 bits
    // otherwise, i.e. sKb as parsed
    out[2 + ra.kdst[c]] = sKb[c];
  }
  if (threadIdx.x == 0) {
    out[0] = (uint64_t)s_n;
    out[1] = 0;
  }
}

// Position after the last '\n' in [0, n), or 0 when there is none; one
// workgroup scans backwards in SEG-byte windows.
__global__ void k_last_newline(const char* buf, int64_t n, int64_t* out) {
  __shared__ unsigned long long best;
  if (threadIdx.x == 0) best = 0;
  __syncthreads();
  for (int64_t hi = n; hi > 0; hi -= SEG) {
    const int64_t lo = hi > SEG ? hi - SEG : 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x)
      if (buf[i] == '\n') atomicMax(&best, (unsigned long long)(i + 1));
    __syncthreads();
    if (best > 0) break;
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = (int64_t)best;
}

// Newlines in a sample of [0, n), 64 windows: the 64 equal parts of it up
// to 1 MiB, else 16 KiB at the start of each 64th.  Workgroup k (1024
// threads, 16 bytes each, all loads in flight at once) writes the count of
// window k to out[k].  The chunk's mean line length sets the fused kernel's
// segment size.
constexpr int kDensWin = 64;
constexpr int kDensBytes = 16 << 10;
__global__ __launch_bounds__(1024) void k_line_density(const char* buf, int64_t n, int64_t* out) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  const int k = blockIdx.x;
  const bool all = n <= (int64_t)kDensWin * kDensBytes;
  const int64_t lo = all ? n * k / kDensWin : (n / kDensWin) * k;
  const int64_t hi = all ? n * (k + 1) / kDensWin : lo + kDensBytes;
  const int64_t i0 = lo + 16 * (int64_t)threadIdx.x;
  int c = 0;
#pragma unroll
  for (int u = 0; u < 16; ++u) c += (i0 + u < hi && buf[i0 + u] == '\n') ? 1 : 0;
  atomicAdd(&cnt, c);
  __syncthreads();
  if (threadIdx.x == 0) out[k] = cnt;
}

// ---- CSV -> fixed-width binary rows ------------------------------------------

// Line starts per segment ([s0, s1) as in k_text), read from global memory.
__global__ __launch_bounds__(kThreads) void k_seg_lines(const char* buf, int64_t nend, int64_t* counts) {
  __shared__ int s_sum[kThreads / 64];
  const int64_t s0 = (int64_t)blockIdx.x * SEG;
  const int64_t s1 = min(s0 + (int64_t)SEG, nend);
  // newlines at m in [max(s0 - 1, 0), s1 - 1) start the lines after s0
  const int64_t ma = s0 > 0 ? s0 - 1 : 0, mz = s1 - 1;
  int mine = 0;
  for (int64_t m = ma + threadIdx.x; m < mz; m += kThreads) mine += buf[m] == '\n';
  if (s0 == 0 && threadIdx.x == 0 && s1 > 0) ++mine;  // the stream's first line
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) mine += __shfl_down(mine, d, 64);
  if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int k = 0; k < kThreads / 64; ++k) t += s_sum[k];
    counts[blockIdx.x] = t;
  }
}

// In-place exclusive scan of n counts (one workgroup); total -> counts[n].
__global__ __launch_bounds__(1024) void k_scan_counts(int64_t* counts, int64_t n) {
  __shared__ int64_t s_part[1024];
  __shared__ int64_t s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < n; b0 += 1024) {
    const int64_t i = b0 + threadIdx.x;
    const int64_t v = i < n ? counts[i] : 0;
    s_part[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
      const int64_t y = threadIdx.x >= (unsigned)d ? s_part[threadIdx.x - d] : 0;
      __syncthreads();
      s_part[threadIdx.x] += y;
      __syncthreads();
    }
    const int64_t excl = s_carry + s_part[threadIdx.x] - v;
    if (i < n) counts[i] = excl;
    __syncthreads();
    if (threadIdx.x == 1023) s_carry += s_part[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[n] = s_carry;
}

struct ConvArgs {
  Args t;                    // text, its line limit, p, integer mask, offsets, status
  const int64_t* seg_base;   // first output row of each segment
  char* out[16];             // column c of row r at out[c] + r * stride[c]
  int64_t stride[16];
  int32_t dtype[16];         // STATS_I32 / STATS_I64 / STATS_F64
};

// One parsed field into its binary column; false when the value does not fit
// the column's type (an integer beyond int32, or beyond 2^53 for FP64).
__device__ inline bool store_field(const ConvArgs& a, int c, int64_t r, uint64_t bits, bool is_int) {
  char* dst = a.out[c] + r * a.stride[c];
  switch (a.dtype[c]) {
    case STATS_I32: {
      const int64_t v = (int64_t)bits;
      if (v < INT32_MIN || v > INT32_MAX) return false;
      *(int32_t*)dst = (int32_t)v;
      return true;
    }
    case STATS_I64: *(int64_t*)dst = (int64_t)bits; return true;
    default: {
      if (is_int) {
        const int64_t v = (int64_t)bits;
        if (v > ((int64_t)1 << 53) || v < -((int64_t)1 << 53)) return false;
        *(double*)dst = (double)v;
      } else {
        *(uint64_t*)dst = bits;
      }
      return true;
    }
  }
}

template <int P>
__global__ __launch_bounds__(kThreads) void k_text_convert(ConvArgs a) {
  __shared__ __attribute__((aligned(16))) unsigned char s_buf[STAGE_PADDED];
  __shared__ unsigned short s_ls[MAXLS];
  __shared__ int s_wsum[kThreads / 64];
  const Args& t = a.t;
  const int64_t s0 = (int64_t)blockIdx.x * SEG;
  const int64_t s1 = min(s0 + (int64_t)SEG, t.nend);
  const int64_t w0r = s0 >= 16 ? s0 - 16 : 0;  // first stream byte staged
  const int64_t w1 = min(s1 + (int64_t)MAXLINE, t.nbytes);
  // w0: stream offset of LDS position 0 (the staging origin is aligned)
  const int64_t w0 = w0r - stage_text(t.buf, w0r, (int)(w1 - w0r), s_buf);
  const int n = (int)(w1 - w0);
  __syncthreads();
  const Stage S{s_buf, w0, n, (int)(min(t.nend, w0 + (int64_t)n) - w0)};
  const int s0r = (int)(s0 - w0), s1r = (int)(s1 - w0);
  Cur C(S);
  int c0, c1, before;
  const int total = line_starts(s_buf, w0, s0r, s1r, SLICE, s_ls, s_wsum, &c0, &c1, &before);
  const int64_t base = a.seg_base[blockIdx.x];
  int first_bad = INT32_MAX;
  // parses line L (k-th of the segment) into output row base + k
  auto put_line = [&](int L, int k) -> int {
    uint64_t row[P];
    int bad_at = INT32_MAX;
    const int end = parse_line_p<P>(t, C, L, row, &bad_at);
    if (end < 0) {
      first_bad = min(first_bad, L);  // reported by the line's first byte
      return -end;  // (-1 - e) + 1: past the offending line
    }
#pragma unroll
    for (int c = 0; c < P; ++c)
      if (!store_field(a, c, base + k, row[c], (t.intmask >> c) & 1u)) first_bad = min(first_bad, L);
    return end + 1;
  };
  if (total <= MAXLS) {
    for (int k = threadIdx.x; k < total; k += kThreads) (void)put_line((int)s_ls[k], k);
  } else {
    // too many lines for the table: each thread walks its own slice
    int L = c0, k = before;
    if (w0 + L > 0)
      while (L < c1 && C.at(L - 1) != '\n') ++L;
    while (L < c1) L = put_line(L, k++);
  }
  if (first_bad != INT32_MAX) {
    atomicMin(&t.status->parse_off, (unsigned long long)(t.base_off + w0 + first_bad));
    atomicOr(&t.status->bits, ST_PARSE);
  }
}

template <int P>
void launch_convert_p(const ConvArgs& a, int64_t nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_text_convert<P>, dim3((unsigned)nblocks), dim3(kThreads), 0, s, a);
}

template <int P>
void launch_text_p(const Args& a, int64_t nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_text<P>, dim3((unsigned)nblocks), dim3(kThreads), 0, s, a);
}

}  // namespace text

using namespace text;

// Segment size of the fused kernel for lines of mean length ell bytes.  A
// workgroup parses its lines 256 at a time (one per thread); the last round
// runs with the lanes that still have a line, and the workgroup holds its
// compute unit until then, so a segment whose line count just passes a
// multiple of 256 wastes most of a round.  Each multiple of 4096 from 16 KiB
// to SEG_MAX is scored as the filled share of its rounds (its count taken 3 %
// high for the spread between segments) times seg / (seg + 4.8 KiB) (the
// fixed cost of a workgroup: the staged overlap, the line table, the final
// sums and the record), halved when the lines would overflow the line table
// (MAXLS; its fallback scans slices); the best one is used.  Without a
// measurement: 32 KiB.
static int pick_text_seg(double ell) {
  if (!(ell > 0.0)) return SEG;
  int best = SEG;
  double best_score = -1.0;
  for (int seg = 16 << 10; seg <= SEG_MAX; seg += 4096) {
    const double lines = seg / ell;
    const double rounds = std::ceil(lines * 1.03 / kThreads);
    const double score = lines / (rounds * kThreads) * seg / (seg + 4915.0) * (lines * 1.03 <= MAXLS ? 1.0 : 0.5);
    if (score > best_score) {
      best_score = score;
      best = seg;
    }
  }
  return best;
}

static int text_launch(stats_ctx* h, const char* dbuf, int64_t nbytes, int64_t nend, int64_t base_off) {
  const int p = h->p;
  const int seg = pick_text_seg(h->text_ell);
  const int64_t nblocks = (nend + seg - 1) / seg;
  if (nblocks == 0) return STATS_OK;
  const int64_t W = rec_words(p);
  // block records, then the slice totals of the merge
  const int64_t part_words = merge_slice_words(nblocks, p);
  int rc = ensure_dev(h, (void**)&h->rec, &h->rec_cap, (size_t)((nblocks * W + part_words) * 8));
  if (rc) return rc;
  Args a;
  memset(&a, 0, sizeof a);
  a.buf = dbuf;
  a.nbytes = nbytes;
  a.nend = nend;
  a.p = p;
  a.base_off = base_off;
  a.seg = seg;
  a.status = h->status_dev;
  uint32_t intmask = 0;
  for (int c = 0; c < p; ++c)
    if (h->intf[c]) intmask |= 1u << c;
  a.intmask = intmask;
  acc::Args& x = a.acc;
  for (int c = 0; c < 16; ++c) {
    x.dtype[c] = (c < p && h->intf[c]) ? STATS_I64 : STATS_F64;
    x.kdst[c] = (int8_t)(c < p ? c : 0);
  }
  x.intmask = intmask;
  x.chkmask = 0;
  int e = p;
  for (int i = 0; i < p; ++i) x.dst[i] = (int16_t)i;
  for (int i = 0; i < p; ++i)
    for (int j = i; j < p; ++j) x.dst[e++] = (int16_t)(p + tri(p, i, j));
  x.rec = h->rec;
  {
    Timer t;
    t.begin(h, STATS_K_TEXT);
    switch (p) {
#define ST_CASE(PP) \
  case PP: launch_text_p<PP>(a, nblocks, h->stream); break;
      ST_CASE(1) ST_CASE(2) ST_CASE(3) ST_CASE(4) ST_CASE(5) ST_CASE(6) ST_CASE(7) ST_CASE(8)
      ST_CASE(9) ST_CASE(10) ST_CASE(11) ST_CASE(12) ST_CASE(13) ST_CASE(14) ST_CASE(15) ST_CASE(16)
#undef ST_CASE
    }
    t.end();
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return hip_fail(h, err, "text kernel launch");
  {
    Timer t;
    t.begin(h, STATS_K_MERGE);
    launch_merge_records(h->rec, nblocks, p, h->intf_dev, h->state[h->cur], h->state[h->cur ^ 1], h->status_dev, h->stream,
                         part_words ? h->rec + nblocks * W : nullptr);
    t.end();
  }
  err = hipGetLastError();
  if (err != hipSuccess) return hip_fail(h, err, "merge kernel launch");
  h->cur ^= 1;
  return STATS_OK;
}

}  // namespace st

using namespace st;

extern "C" int stats_accumulate_text(stats_ctx* h, const char* buf, int64_t nbytes, int32_t mem_kind,
                                     int32_t is_last, int64_t* bytes_consumed) {
  if (!h) return fail(STATS_E_ARG, "handle is NULL");
  if (h->poisoned) return fail(STATS_E_STATE, "handle is poisoned by an earlier HIP error");
  if (h->ngroups) return fail(STATS_E_STATE, "groups handle: text input is not supported");
  if (h->flags & STATS_CFG_PAIRWISE) return fail(STATS_E_STATE, "pairwise handle: text input is not supported");
  if (!bytes_consumed) return fail(STATS_E_ARG, "bytes_consumed is NULL");
  *bytes_consumed = 0;
  if (nbytes < 0) return fail(STATS_E_ARG, "nbytes < 0");
  if (h->p > 16) return fail(STATS_E_ARG, "text ingest supports p <= 16");
  if (nbytes == 0) return STATS_OK;
  if (!buf) return fail(STATS_E_ARG, "buf is NULL");
  DeviceGuard g(h->device);
  if (!g.ok) return fail(STATS_E_HIP, "hipSetDevice failed");
  const char* dbuf = buf;
  hipError_t e;
  if (mem_kind == STATS_MEM_HOST || mem_kind == STATS_MEM_HOST_PINNED) {
    int rc = ensure_dev(h, &h->aux_dev, &h->aux_cap, (size_t)nbytes);
    if (rc) return rc;
    e = hipMemcpyAsync(h->aux_dev, buf, (size_t)nbytes, hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "copying text to the device");
    dbuf = (const char*)h->aux_dev;
  } else if (mem_kind != STATS_MEM_DEVICE) {
    return fail(STATS_E_ARG, "unknown mem_kind");
  }
  int64_t nend = nbytes;
  // the last line end of a chunk that is not the last one, and the chunk's
  // line density (every chunk that waits for the first anyway, and a last
  // chunk when nothing was measured before)
  if (!is_last || !(h->text_ell > 0.0)) {
    int rc = ensure_dev(h, (void**)&h->raw_out, &h->raw_cap, 8 * (1 + kDensWin));
    if (rc) return rc;
    int64_t* ro = (int64_t*)h->raw_out;
    if (!is_last) hipLaunchKernelGGL(k_last_newline, dim3(1), dim3(1024), 0, h->stream, dbuf, nbytes, ro);
    hipLaunchKernelGGL(k_line_density, dim3(kDensWin), dim3(1024), 0, h->stream, dbuf, nbytes, ro + 1);
    e = hipGetLastError();
    int64_t hv[1 + kDensWin];
    hv[0] = nbytes;
    if (e == hipSuccess)
      e = hipMemcpyAsync(is_last ? hv + 1 : hv, is_last ? ro + 1 : ro, 8 * (is_last ? kDensWin : 1 + kDensWin),
                         hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "finding the last line end");
    nend = hv[0];
    int64_t lines = 0;
    for (int k = 1; k <= kDensWin; ++k) lines += hv[k];
    const int64_t counted = nbytes <= (int64_t)kDensWin * kDensBytes ? nbytes : (int64_t)kDensWin * kDensBytes;
    if (lines > 0) h->text_ell = (double)counted / (double)lines;
  }
  const int64_t base_off = h->text_offset;
  int rc = text_launch(h, dbuf, nbytes, nend, base_off);
  if (rc) return rc;
  if (mem_kind != STATS_MEM_DEVICE) {
    e = hipStreamSynchronize(h->stream);  // the staging copy may be reused by the next call
    if (e != hipSuccess) return hip_fail(h, e, "text ingest");
  }
  h->text_offset += nend;
  *bytes_consumed = nend;
  return STATS_OK;
}

extern "C" int stats_text_to_binary(stats_ctx* h, const char* buf, int64_t nbytes, int32_t mem_kind,
                                    int32_t is_last, void* const* out_planes, int64_t max_rows,
                                    int64_t* rows_out, int64_t* bytes_consumed) {
  if (!h) return fail(STATS_E_ARG, "handle is NULL");
  if (h->poisoned) return fail(STATS_E_STATE, "handle is poisoned by an earlier HIP error");
  if (h->ngroups) return fail(STATS_E_STATE, "groups handle: text conversion is not supported");
  if (!bytes_consumed || !rows_out) return fail(STATS_E_ARG, "rows_out or bytes_consumed is NULL");
  *bytes_consumed = 0;
  *rows_out = 0;
  if (nbytes < 0 || max_rows < 0) return fail(STATS_E_ARG, "nbytes or max_rows < 0");
  const int p = h->p;
  if (p > 16) return fail(STATS_E_ARG, "text conversion supports p <= 16");
  for (int c = 0; c < p; ++c) {
    const stats_column& col = h->cols[c];
    if (col.dtype == STATS_F32) return fail(STATS_E_ARG, "text conversion writes I32, I64 or F64 columns");
    if (!h->intf[c] && col.dtype != STATS_F64)
      return fail(STATS_E_ARG, "a decimal (non-integer) column must be stored as F64");
  }
  if (nbytes == 0) return STATS_OK;
  if (!buf || !out_planes) return fail(STATS_E_ARG, "buf or out_planes is NULL");
  for (int c = 0; c < p; ++c)
    if (!out_planes[h->cols[c].plane]) return fail(STATS_E_ARG, "an output plane is NULL");
  DeviceGuard g(h->device);
  if (!g.ok) return fail(STATS_E_HIP, "hipSetDevice failed");
  const char* dbuf = buf;
  hipError_t e;
  if (mem_kind == STATS_MEM_HOST || mem_kind == STATS_MEM_HOST_PINNED) {
    int rc = ensure_dev(h, &h->aux_dev, &h->aux_cap, (size_t)nbytes);
    if (rc) return rc;
    e = hipMemcpyAsync(h->aux_dev, buf, (size_t)nbytes, hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "copying text to the device");
    dbuf = (const char*)h->aux_dev;
  } else if (mem_kind != STATS_MEM_DEVICE) {
    return fail(STATS_E_ARG, "unknown mem_kind");
  }
  const int64_t nseg_max = (nbytes + SEG - 1) / SEG;
  // scratch: per-segment counts / first rows (nseg + 1), the last line end,
  // and a status word of its own (the handle's statistics are not touched)
  const size_t cnt_bytes = (size_t)(nseg_max + 1) * 8;
  const size_t need = (cnt_bytes + 255) / 256 * 256 + 256;
  int rc = ensure_dev(h, &h->conv_dev, &h->conv_cap, need);
  if (rc) return rc;
  int64_t* counts = (int64_t*)h->conv_dev;
  char* tailp = (char*)h->conv_dev + (cnt_bytes + 255) / 256 * 256;
  int64_t* nend_dev = (int64_t*)tailp;
  DevStatus* cst = (DevStatus*)(tailp + 64);
  static const DevStatus init = {0u, 0u, ~0ull};
  e = hipMemcpyAsync(cst, &init, sizeof init, hipMemcpyHostToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "clearing the conversion status");
  int64_t nend = nbytes;
  if (!is_last) {
    hipLaunchKernelGGL(k_last_newline, dim3(1), dim3(1024), 0, h->stream, dbuf, nbytes, nend_dev);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&nend, nend_dev, 8, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "finding the last line end");
  }
  const int64_t nseg = (nend + SEG - 1) / SEG;
  if (nseg == 0) return STATS_OK;
  hipLaunchKernelGGL(k_seg_lines, dim3((unsigned)nseg), dim3(kThreads), 0, h->stream, dbuf, nend, counts);
  e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, h->stream, counts, nseg);
    e = hipGetLastError();
  }
  int64_t total = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&total, counts + nseg, 8, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "counting lines");
  if (total > max_rows)
    return fail(STATS_E_ARG, "the chunk holds " + std::to_string(total) + " lines, the output " +
                                 std::to_string(max_rows) + " rows");
  ConvArgs a;
  memset(&a, 0, sizeof a);
  a.t.buf = dbuf;
  a.t.nbytes = nbytes;
  a.t.nend = nend;
  a.t.p = p;
  a.t.base_off = h->text_offset;
  a.t.status = cst;
  for (int c = 0; c < p; ++c)
    if (h->intf[c]) a.t.intmask |= 1u << c;
  a.seg_base = counts;
  for (int c = 0; c < p; ++c) {
    const stats_column& col = h->cols[c];
    a.out[c] = (char*)out_planes[col.plane] + col.byte_offset;
    a.stride[c] = h->row_stride[col.plane];
    a.dtype[c] = col.dtype;
  }
  switch (p) {
#define ST_CASE(PP) \
  case PP: launch_convert_p<PP>(a, nseg, h->stream); break;
    ST_CASE(1) ST_CASE(2) ST_CASE(3) ST_CASE(4) ST_CASE(5) ST_CASE(6) ST_CASE(7) ST_CASE(8)
    ST_CASE(9) ST_CASE(10) ST_CASE(11) ST_CASE(12) ST_CASE(13) ST_CASE(14) ST_CASE(15) ST_CASE(16)
#undef ST_CASE
  }
  e = hipGetLastError();
  DevStatus st{};
  if (e == hipSuccess) e = hipMemcpyAsync(&st, cst, sizeof st, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "text conversion");
  h->text_offset += nend;
  if (st.bits & ST_PARSE)
    return fail(STATS_E_PARSE, "malformed or out-of-range field in the line starting at byte offset " +
                                   std::to_string((unsigned long long)st.parse_off));
  *rows_out = total;
  *bytes_consumed = nend;
  return STATS_OK;
}
