// Four-step splits of the Bluestein lengths, as measured on MI355X by
// paper_1711_05152_amd/tune_fft.py (which rewrites this file): kTunedSplit[dtype][lgN] is lgN1 of
// 2^lgN = 2^lgN1 * 2^(lgN - lgN1) for dtype 0 = complex64, 1 = complex128; -1 keeps the rule.
#pragma once
#include <stdint.h>
static const int8_t kTunedSplit[2][25] = {
    {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, 7, 8, 8, -1, -1, -1, -1, -1, -1, -1, -1, -1},
    {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, 7, 8, 8, -1, -1, -1, -1, -1, -1, -1, -1, -1},
};
// Stage-2 variants (bit 0: radix schedule of orders 3 / 2; bit 1: 4096-element row tiles; bit 2:
// 8 values per thread) chosen by the same tuner: kTunedP2[dtype][lgN] for the split of kTunedSplit;
// -1 keeps variant 0.
static const int8_t kTunedP2[2][25] = {
    {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, 6, 6, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1},
    {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, 6, 6, -1, -1, 4, -1, -1, -1, -1, -1, -1, -1},
};
// Bluestein length classes 2^lg whose lattices take 3 * 2^(lg - 2) when all of them fit, chosen by
// the same tuner (1: the factor-3 length measured faster; 0 or -1: powers of two).
static const int8_t kTunedSmooth[2][25] = {
    {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, 1, 1, 1, 1, -1, 1, 1},
};
