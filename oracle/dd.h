/*
 * Double-double arithmetic for the CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the GPU library includes this file and
 * nothing here is shared with it.
 *
 * A value is an unevaluated sum hi + lo with |lo| <= ulp(hi)/2. The building
 * blocks are the error-free transformations of Sec. 2.2 of the paper:
 * Knuth's TwoSum (x = fl(a+b), y = a + b - x exactly) and the pair arithmetic
 * that adds a double-word number while dropping part of the low word. The
 * exact product uses a fused multiply-add: for p = fl(a*b), a*b - p is
 * representable and fma(a, b, -p) returns it exactly.
 *
 * This file must be compiled with -ffp-contract=off: the compiler may not
 * merge or reorder any of the operations below.
 */
#ifndef ORACLE_DD_H
#define ORACLE_DD_H

#include <math.h>

typedef struct { double hi, lo; } dd_t;

/* Knuth's TwoSum: s + e == a + b exactly, s = fl(a + b). */
static inline dd_t two_sum(double a, double b)
{
    double s = a + b;
    double z = s - a;
    double e = (a - (s - z)) + (b - z);
    dd_t r = { s, e };
    return r;
}

/* Dekker's FastTwoSum, valid when |a| >= |b| (or a == 0). */
static inline dd_t fast_two_sum(double a, double b)
{
    double s = a + b;
    double e = b - (s - a);
    dd_t r = { s, e };
    return r;
}

/* p + e == a * b exactly (no underflow), p = fl(a * b). */
static inline dd_t two_prod(double a, double b)
{
    double p = a * b;
    double e = fma(a, b, -p);
    dd_t r = { p, e };
    return r;
}

static inline dd_t dd_from(double a) { dd_t r = { a, 0.0 }; return r; }
static inline dd_t dd_neg(dd_t a) { dd_t r = { -a.hi, -a.lo }; return r; }

/* (a.hi + a.lo) + (b.hi + b.lo): TwoSum of both words, then renormalise. */
static inline dd_t dd_add(dd_t a, dd_t b)
{
    dd_t s = two_sum(a.hi, b.hi);
    dd_t t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return fast_two_sum(s.hi, s.lo);
}

static inline dd_t dd_sub(dd_t a, dd_t b) { return dd_add(a, dd_neg(b)); }

/* Pair arithmetic of Sec. 2.2: a + (b.hi + b.lo) with the low word of the
 * result taken as fl(b.lo + t). Used for accumulations where every addend is
 * small relative to the running sum or exact. */
static inline dd_t dd_add_pair(dd_t a, dd_t b)
{
    dd_t s = two_sum(a.hi, b.hi);
    s.lo = s.lo + (a.lo + b.lo);
    return fast_two_sum(s.hi, s.lo);
}

static inline dd_t dd_mul(dd_t a, dd_t b)
{
    dd_t p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return fast_two_sum(p.hi, p.lo);
}

static inline dd_t dd_mul_d(dd_t a, double b)
{
    dd_t p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return fast_two_sum(p.hi, p.lo);
}

/* a / b by long division with three partial quotients. */
static inline dd_t dd_div(dd_t a, dd_t b)
{
    double q1 = a.hi / b.hi;
    dd_t r = dd_sub(a, dd_mul_d(b, q1));
    double q2 = r.hi / b.hi;
    r = dd_sub(r, dd_mul_d(b, q2));
    double q3 = r.hi / b.hi;
    dd_t q = fast_two_sum(q1, q2);
    return dd_add(q, dd_from(q3));
}

/* sqrt(a) for a >= 0: one Newton step from the FP64 root. */
static inline dd_t dd_sqrt(dd_t a)
{
    if (a.hi <= 0.0) return dd_from(0.0);
    double x = sqrt(a.hi);
    dd_t x2 = two_prod(x, x);
    dd_t r = dd_sub(a, x2);
    double corr = r.hi / (2.0 * x);
    return fast_two_sum(x, corr);
}

static inline double dd_abs_hi(dd_t a) { return fabs(a.hi); }

#endif
