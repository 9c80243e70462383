// Runtime dispatch over the compiled (dimension, degree, equation) set:
// D in {2, 3}, p in {1..4}, equation in {Poisson, Euler, Navier-Stokes}.
// The body sees constexpr D, P, EQ and must return a hipError_t.
#pragma once

#define LDG_CASE(D_, P_, EQ_, ...)            \
  case D_ * 100 + P_ * 10 + EQ_: {            \
    constexpr int D = D_, P = P_, EQ = EQ_;   \
    __VA_ARGS__                               \
  }
#define LDG_DISPATCH(DC, ...)                                                                        \
  switch ((DC).D * 100 + (DC).P * 10 + (DC).EQ) {                                                    \
    LDG_CASE(2, 1, 0, __VA_ARGS__) LDG_CASE(2, 2, 0, __VA_ARGS__) LDG_CASE(2, 3, 0, __VA_ARGS__)     \
    LDG_CASE(2, 4, 0, __VA_ARGS__) LDG_CASE(2, 1, 1, __VA_ARGS__) LDG_CASE(2, 2, 1, __VA_ARGS__)     \
    LDG_CASE(2, 3, 1, __VA_ARGS__) LDG_CASE(2, 4, 1, __VA_ARGS__) LDG_CASE(2, 1, 2, __VA_ARGS__)     \
    LDG_CASE(2, 2, 2, __VA_ARGS__) LDG_CASE(2, 3, 2, __VA_ARGS__) LDG_CASE(2, 4, 2, __VA_ARGS__)     \
    LDG_CASE(3, 1, 0, __VA_ARGS__) LDG_CASE(3, 2, 0, __VA_ARGS__) LDG_CASE(3, 3, 0, __VA_ARGS__)     \
    LDG_CASE(3, 4, 0, __VA_ARGS__) LDG_CASE(3, 1, 1, __VA_ARGS__) LDG_CASE(3, 2, 1, __VA_ARGS__)     \
    LDG_CASE(3, 3, 1, __VA_ARGS__) LDG_CASE(3, 4, 1, __VA_ARGS__) LDG_CASE(3, 1, 2, __VA_ARGS__)     \
    LDG_CASE(3, 2, 2, __VA_ARGS__) LDG_CASE(3, 3, 2, __VA_ARGS__) LDG_CASE(3, 4, 2, __VA_ARGS__)     \
    default:                                                                                         \
      return hipErrorInvalidValue;                                                                   \
  }
