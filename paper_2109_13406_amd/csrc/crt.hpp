// crt.hpp -- host-side constants of the modular (Chinese-remainder) split
// form: the moduli, the integer grid width P, and the per-modulus constants
// its residue and reconstruction kernels take by value.  Internal to libmpdd.
//
// The form (after the integer modular emulation of a floating-point matrix
// product by Ozaki, Uchino and Imamura, "Ozaki scheme II", 2025, applied to
// dd operands): each row of op(A) and column of op(B) is rounded to integers
// on a grid of P bits below its largest |hi| (x' = rint(zh) + rint((zh -
// rint(zh)) + zl), z = x 2^(P - sigma)); the integers are reduced modulo
// `count` pairwise coprime moduli <= 256 to balanced residues that fit int8;
// one exact INT8 product per modulus; the exact integer product is rebuilt
// from the residues of its entries by Chinese remaindering and rounded to dd.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <cmath>
#include <cstdint>
#include <mutex>

namespace mpdd {

constexpr int CRT_MAX_MODULI = 32;   // moduli a call may use
constexpr int CRT_MAX_BITS = 104;    // widest grid: the chunks of x' stay below 2^53
constexpr int CRT_LIMB_BITS = 39;    // reconstruction limbs: 32 * 2^7 * 2^39 < 2^52
constexpr int CRT_MAX_LIMBS = 7;     // 7 * 39 >= 257 bits > bits of 256^32
constexpr int64_t CRT_MAX_K = ((int64_t)1 << 17) - 1;   // k 128^2 < 2^31

// Residue kernel constants, per modulus t: m, 1/m and 2^26, 2^52, 2^78
// modulo m (x' = u1 2^78 + u0 2^52 + w1 2^26 + w0 in 26-bit chunks).
struct CrtResidueConsts {
  double m[CRT_MAX_MODULI], minv[CRT_MAX_MODULI];
  double c26[CRT_MAX_MODULI], c52[CRT_MAX_MODULI], c78[CRT_MAX_MODULI];
};

// Reconstruction constants in 26-bit limbs (the qd form, whose three
// sub-products are recombined limb-wise at offsets of 104 = 4 x 26 bits).
constexpr int CRT_LIMB26 = 26;
constexpr int CRT_MAX_LIMBS26 = 10;     // 10 * 26 >= 257
struct CrtCombineConsts26 {
  double w[CRT_MAX_MODULI][CRT_MAX_LIMBS26];
  double ml[CRT_MAX_LIMBS26], g[CRT_MAX_LIMBS26];
};

// The qd form: grid of 208 bits, split at 2^104; its three sub-products
// (each below 2^212 k in magnitude) are recovered when M >= 2^(215 +
// ceil(log2 k)).
constexpr int CRT_QD_GRID_BITS = 208;

// The moduli and their reciprocals, for the products' reduction.
struct CrtModuli {
  double m[CRT_MAX_MODULI], minv[CRT_MAX_MODULI];
};

// Reconstruction constants: the CRT weights W_t = (M/m_t) ((M/m_t)^-1 mod
// m_t) in base-2^39 limbs; the limbs of M; and g_l = 2^(39 l) / M (rounded),
// which estimate the multiple of M to remove.
struct CrtCombineConsts {
  double w[CRT_MAX_MODULI][CRT_MAX_LIMBS];
  double ml[CRT_MAX_LIMBS], g[CRT_MAX_LIMBS];
};

// The moduli: from 256 down, every integer coprime to all the moduli
// already taken (the list is built once per process).
inline const std::array<int, CRT_MAX_MODULI>& crt_moduli_list() {
  static const std::array<int, CRT_MAX_MODULI> list = [] {
    std::array<int, CRT_MAX_MODULI> out{};
    int got = 0;
    for (int m = 256; got < CRT_MAX_MODULI && m >= 2; --m) {
      bool ok = true;
      for (int i = 0; i < got && ok; ++i) {
        int a = m, b = out[i];
        while (b) {
          const int t = a % b;
          a = b;
          b = t;
        }
        ok = (a == 1);
      }
      if (ok) out[got++] = m;
    }
    return out;
  }();
  return list;
}

// The first `count` moduli (count <= CRT_MAX_MODULI).
inline void crt_moduli(int count, int* out) {
  const auto& list = crt_moduli_list();
  for (int t = 0; t < count && t < CRT_MAX_MODULI; ++t) out[t] = list[t];
}

// Unsigned multiword integer, 32-bit words, least significant first (enough
// for the product of 32 moduli <= 256 and a weight below it).
struct CrtBig {
  uint32_t w[10] = {};
  void mul(uint32_t s) {
    uint64_t carry = 0;
    for (uint32_t& x : w) {
      const uint64_t v = (uint64_t)x * s + carry;
      x = (uint32_t)v;
      carry = v >> 32;
    }
  }
  uint32_t divmod(uint32_t s) {        // *this /= s; returns the remainder
    uint64_t rem = 0;
    for (int i = 9; i >= 0; --i) {
      const uint64_t v = (rem << 32) | w[i];
      w[i] = (uint32_t)(v / s);
      rem = v % s;
    }
    return (uint32_t)rem;
  }
  int bits() const {
    for (int i = 9; i >= 0; --i)
      if (w[i]) return 32 * i + 32 - __builtin_clz(w[i]);
    return 0;
  }
  uint64_t field(int pos, int nbits) const {   // bits [pos, pos + nbits), nbits <= 40
    uint64_t v = 0;
    for (int b = 0; b < nbits; ++b) {
      const int q = pos + b;
      if (q < 320 && ((w[q >> 5] >> (q & 31)) & 1u)) v |= (uint64_t)1 << b;
    }
    return v;
  }
  double approx() const {
    double v = 0.0;
    for (int i = 9; i >= 0; --i) v = v * 4294967296.0 + (double)w[i];
    return v;
  }
};

inline CrtBig crt_modulus_product(int count) {
  int ms[CRT_MAX_MODULI];
  crt_moduli(count, ms);
  CrtBig M;
  M.w[0] = 1;
  for (int t = 0; t < count; ++t) M.mul((uint32_t)ms[t]);
  return M;
}

// Bit length of M for 1 .. CRT_MAX_MODULI moduli (built once per process;
// 0 for a count outside that range).
inline int crt_modulus_bits(int count) {
  if (count < 1 || count > CRT_MAX_MODULI) return 0;
  static const std::array<int, CRT_MAX_MODULI + 1> bits = [] {
    std::array<int, CRT_MAX_MODULI + 1> b{};
    for (int c = 1; c <= CRT_MAX_MODULI; ++c) b[c] = crt_modulus_product(c).bits();
    return b;
  }();
  return bits[count];
}

// P: the largest P <= CRT_MAX_BITS with 4 k 2^(2P) <= M (so that every
// entry of the integer product, at most k 2^(2P) in magnitude, lies in
// [-M/4, M/4] and is recovered exactly); 0 when count is out of range or
// no P >= 1 fits.
// A complex product (margin 3) needs 8 k 2^(2P) <= M: its parts are sums of
// two products, at most 2 k 2^(2P) in magnitude.
inline int crt_exponent(int64_t k, int count, int margin = 2) {
  if (count < 1 || count > CRT_MAX_MODULI) return 0;
  int lk = 0;
  while (((int64_t)1 << lk) < k) ++lk;            // ceil(log2 k), k >= 1
  const int fl = crt_modulus_bits(count) - 1;
  int p = (fl - margin - lk);
  p = p >= 0 ? p / 2 : -1;
  if (p > CRT_MAX_BITS) p = CRT_MAX_BITS;
  return p >= 1 ? p : 0;
}

// Moduli count used when the caller passes 0: the fewest whose grid reaches
// CRT_MAX_BITS for this k (CRT_MAX_MODULI if none does).
inline int crt_default_count(int64_t k, int margin = 2) {
  for (int c = 1; c <= CRT_MAX_MODULI; ++c)
    if (crt_exponent(k, c, margin) == CRT_MAX_BITS) return c;
  return CRT_MAX_MODULI;
}

// The constant sets for `count` moduli; returns the number of limbs.
inline int crt_constants_build(int count, CrtResidueConsts* rc, CrtModuli* cm,
                               CrtCombineConsts* cc) {
  int ms[CRT_MAX_MODULI];
  crt_moduli(count, ms);
  const CrtBig M = crt_modulus_product(count);
  const int limbs = (M.bits() + CRT_LIMB_BITS - 1) / CRT_LIMB_BITS;
  auto pow2mod = [](int e, int m) {
    int r = 1 % m;
    for (int i = 0; i < e; ++i) r = (2 * r) % m;
    return r;
  };
  for (int t = 0; t < CRT_MAX_MODULI; ++t) {
    const bool on = t < count;
    const int m = on ? ms[t] : 1;
    rc->m[t] = cm->m[t] = m;
    rc->minv[t] = cm->minv[t] = 1.0 / m;
    rc->c26[t] = on ? pow2mod(26, m) : 0.0;
    rc->c52[t] = on ? pow2mod(52, m) : 0.0;
    rc->c78[t] = on ? pow2mod(78, m) : 0.0;
    for (int l = 0; l < CRT_MAX_LIMBS; ++l) cc->w[t][l] = 0.0;
    if (!on) continue;
    CrtBig Mt = M;
    Mt.divmod((uint32_t)m);                      // exact: m divides M
    CrtBig tmp = Mt;
    const int64_t r = tmp.divmod((uint32_t)m);   // M/m_t mod m_t (coprime to m_t)
    // inverse of r modulo m (extended Euclid)
    int64_t a = r, b = m, x0 = 1, x1 = 0;
    while (b) {
      const int64_t q = a / b, ta = a - q * b, tx = x0 - q * x1;
      a = b;
      b = ta;
      x0 = x1;
      x1 = tx;
    }
    const int64_t inv = ((x0 % m) + m) % m;
    CrtBig W = Mt;
    W.mul((uint32_t)inv);
    for (int l = 0; l < limbs; ++l)
      cc->w[t][l] = (double)W.field(CRT_LIMB_BITS * l, CRT_LIMB_BITS);
  }
  const double minv = 1.0 / M.approx();
  for (int l = 0; l < CRT_MAX_LIMBS; ++l) {
    cc->ml[l] = l < limbs ? (double)M.field(CRT_LIMB_BITS * l, CRT_LIMB_BITS) : 0.0;
    cc->g[l] = l < limbs ? std::ldexp(minv, CRT_LIMB_BITS * l) : 0.0;
  }
  return limbs;
}

inline bool crt_qd_count_ok(int64_t k, int count) {
  if (count < 1 || count > CRT_MAX_MODULI) return false;
  int lk = 0;
  while (((int64_t)1 << lk) < k) ++lk;
  return crt_modulus_bits(count) - 1 >= 215 + lk;
}

inline int crt_qd_default_count(int64_t k) {
  for (int c = 1; c <= CRT_MAX_MODULI; ++c)
    if (crt_qd_count_ok(k, c)) return c;
  return 0;
}

// CRT weights and M in 26-bit limbs for `count` moduli.
inline void crt_constants26_build(int count, CrtCombineConsts26* cc) {
  int ms[CRT_MAX_MODULI];
  crt_moduli(count, ms);
  const CrtBig M = crt_modulus_product(count);
  for (int t = 0; t < CRT_MAX_MODULI; ++t) {
    for (int l = 0; l < CRT_MAX_LIMBS26; ++l) cc->w[t][l] = 0.0;
    if (t >= count) continue;
    const int m = ms[t];
    CrtBig Mt = M;
    Mt.divmod((uint32_t)m);
    CrtBig tmp = Mt;
    const int64_t r = tmp.divmod((uint32_t)m);
    int64_t a = r, b = m, x0 = 1, x1 = 0;
    while (b) {
      const int64_t q = a / b, ta = a - q * b, tx = x0 - q * x1;
      a = b;
      b = ta;
      x0 = x1;
      x1 = tx;
    }
    CrtBig W = Mt;
    W.mul((uint32_t)(((x0 % m) + m) % m));
    for (int l = 0; l < CRT_MAX_LIMBS26; ++l)
      cc->w[t][l] = (double)W.field(CRT_LIMB26 * l, CRT_LIMB26);
  }
  const double minv = 1.0 / M.approx();
  for (int l = 0; l < CRT_MAX_LIMBS26; ++l) {
    cc->ml[l] = (double)M.field(CRT_LIMB26 * l, CRT_LIMB26);
    cc->g[l] = std::ldexp(minv, CRT_LIMB26 * l);
  }
}

// crt_constants / crt_constants26 with each count's constants built once per
// process and copied out afterwards (they depend on the count only; building
// them costs tens of microseconds of host time per call).  A count outside
// 1 .. CRT_MAX_MODULI is built each time, uncached.
inline int crt_constants(int count, CrtResidueConsts* rc, CrtModuli* cm, CrtCombineConsts* cc) {
  struct Entry {
    std::once_flag once;
    int limbs = 0;
    CrtResidueConsts rc;
    CrtModuli cm;
    CrtCombineConsts cc;
  };
  static Entry table[CRT_MAX_MODULI + 1];
  if (count < 1 || count > CRT_MAX_MODULI) return crt_constants_build(count, rc, cm, cc);
  Entry& e = table[count];
  std::call_once(e.once, [&] { e.limbs = crt_constants_build(count, &e.rc, &e.cm, &e.cc); });
  *rc = e.rc;
  *cm = e.cm;
  *cc = e.cc;
  return e.limbs;
}

inline void crt_constants26(int count, CrtCombineConsts26* cc) {
  struct Entry {
    std::once_flag once;
    CrtCombineConsts26 cc;
  };
  static Entry table[CRT_MAX_MODULI + 1];
  if (count < 1 || count > CRT_MAX_MODULI) return crt_constants26_build(count, cc);
  Entry& e = table[count];
  std::call_once(e.once, [&] { crt_constants26_build(count, &e.cc); });
  *cc = e.cc;
}

// Complex modular product (ozaki.hip): P = op(A) op(B) of complex dd
// operands (planes re.hi, re.lo, im.hi, im.lo; op 0 'N', 1 'T', 2 'C') into
// the dd planes (prh, prl) + i (pih, pil), leading dimension m, with three
// residue products per modulus (Re = T1 - T2, Im = T3 - T1 - T2).  k >= 1.
int ozaki_crt_cgemm(const void* opts, int opa, int opb, int64_t m, int64_t n, int64_t k,
                    const double* const* a, int64_t lda, const double* const* b, int64_t ldb,
                    double* prh, double* prl, double* pih, double* pil, hipStream_t st,
                    hipMemPool_t pool);

// qd modular product (ozaki.hip): C = alpha op(A) op(B) + beta C on qd
// planes (x0..x3), three residue products per modulus (Karatsuba on the
// 2^104 split).  k >= 1, alpha != 0.
int ozaki_crt_qgemm(const void* opts, bool ta, bool tb, int64_t m, int64_t n, int64_t k,
                    const double* alpha, const double* const* a, int64_t lda,
                    const double* const* b, int64_t ldb, const double* beta, int beta_zero,
                    double* const* c, int64_t ldc, hipStream_t st, hipMemPool_t pool);

}  // namespace mpdd
