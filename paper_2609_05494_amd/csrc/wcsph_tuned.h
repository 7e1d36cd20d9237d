// Scan shapes of the pair pass. The tuner (paper_2609_05494_amd/autotune.py)
// rewrites this file with its measured table; until it has been run on the
// current kernels the shape is the one chosen by hand: C2, the walk along
// each own row unrolled twice measured 89.6 us per step against 90.3 us
// without unrolling (one MI355X, interleaved runs).
// A shape given on the command line (-DUCAP=... when the tuner builds its
// variants) takes precedence over the one recorded here.
#pragma once
#ifndef UCAP
#define UCAP 128
#endif
#ifndef LCAP
#define LCAP 16
#endif
#ifndef RU
#define RU 2
#endif
