// Exact tier (host): verdict of one element in integer arithmetic.
#pragma once
#include <stdint.h>

namespace hexval {
// pts: 8 points (Appendix A order) x 3 coordinates.  Returns 0 INVALID,
// 1 VALID, 2 UNDECIDED, 3 BAD_INPUT (non-finite coordinate).
uint8_t exact_verdict(const double pts[24], int max_depth);
// Corner-only test in integer arithmetic: 1 when the 8 corner values of J
// are all > 0, else 0; 3 for a non-finite coordinate.
uint8_t exact_corner_test(const double pts[24]);
// Linear quadrangle (4 points x 2 coordinates) in integer arithmetic: 1 when
// the four corner values of J are > 0, else 0; 3 for a non-finite coordinate.
uint8_t exact_quad(const double pts[8]);
}
