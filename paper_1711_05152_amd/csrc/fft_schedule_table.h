// Four-step splits of the Bluestein lengths, as measured on MI355X by
// paper_1711_05152_amd/tune_fft.py (which rewrites this file): kTunedSplit[dtype][lgN] is lgN1 of
// 2^lgN = 2^lgN1 * 2^(lgN - lgN1) for dtype 0 = complex64, 1 = complex128; -1 keeps the rule.
#pragma once
#include <stdint.h>
static const int8_t kTunedSplit[2][25] = {
    {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, 8, -1, -1, -1, -1, -1, -1, -1, -1, -1},
    {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, 5, -1, 8, -1, -1, -1, -1, -1, -1, -1, -1, -1},
};
