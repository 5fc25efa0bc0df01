// Compile-time strings: a fixed-size character array whose length is part of
// its type, concatenated with `+` in constant expressions, plus the decimal
// text of a compile-time integer.  The kernel-source generator builds the
// whole text of a kernel from an expression's type with these, so the text
// is a constant of the program (Sec. 3: the library emits each kernel's
// source at compile time with such a compile-time character array and
// compile-time concatenation).
#pragma once

#include <stddef.h>

namespace fx {

template <size_t N> struct cstr {
  char c[N + 1];
  static constexpr size_t size = N;
  constexpr cstr() : c{} {}
  constexpr cstr(const char (&a)[N + 1]) : c{} {
    for (size_t i = 0; i < N; ++i) c[i] = a[i];
  }
  constexpr const char* data() const { return c; }
  constexpr char operator[](size_t i) const { return c[i]; }
};
template <size_t M> cstr(const char (&)[M]) -> cstr<M - 1>;

template <size_t A, size_t B> constexpr cstr<A + B> operator+(const cstr<A>& a, const cstr<B>& b) {
  cstr<A + B> r;
  for (size_t i = 0; i < A; ++i) r.c[i] = a.c[i];
  for (size_t i = 0; i < B; ++i) r.c[A + i] = b.c[i];
  return r;
}
template <size_t A, size_t B> constexpr auto operator+(const cstr<A>& a, const char (&b)[B]) {
  return a + cstr<B - 1>(b);
}
template <size_t A, size_t B> constexpr auto operator+(const char (&a)[A], const cstr<B>& b) {
  return cstr<A - 1>(a) + b;
}

constexpr size_t decimal_digits(long long v) {
  size_t d = v < 0 ? 2 : 1;
  for (unsigned long long u = v < 0 ? 0ull - (unsigned long long)v : (unsigned long long)v; u >= 10;
       u /= 10)
    ++d;
  return d;
}

// The decimal text of V.
template <long long V> constexpr auto num() {
  constexpr size_t D = decimal_digits(V);
  cstr<D> r;
  unsigned long long u = V < 0 ? 0ull - (unsigned long long)V : (unsigned long long)V;
  for (size_t i = D; i-- > (V < 0 ? 1 : 0);) {
    r.c[i] = (char)('0' + u % 10);
    u /= 10;
  }
  if (V < 0) r.c[0] = '-';
  return r;
}

// Does `s` contain `t` (compile-time search; for tests of the emitted text)?
template <size_t N, size_t M> constexpr bool contains(const cstr<N>& s, const char (&t)[M]) {
  if (M - 1 > N) return false;
  for (size_t i = 0; i + (M - 1) <= N; ++i) {
    size_t k = 0;
    while (k < M - 1 && s.c[i + k] == t[k]) ++k;
    if (k == M - 1) return true;
  }
  return false;
}

}  // namespace fx
