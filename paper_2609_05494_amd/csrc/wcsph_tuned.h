// Scan shapes of the pair pass, written by paper_2609_05494_amd/autotune.py.
// Workload C2, 1000 timed steps; ms per step of every shape:
//   u128_l16_p4: 0.0910
//   u192_l16_p4: 0.0912
//   u128_l24_p4: 0.0917
//   u192_l24_p4: 0.0925
//   u192_l24_p8: 0.0942
//   u128_l24_p8: 0.0943
//   u256_l24_p8: 0.0949
//   u256_l24_p4: 0.0952
//   u256_l16_p4: 0.0952
//   u192_l16_p8: 0.0993
//   u128_l16_p8: 0.0995
//   u256_l16_p8: 0.1006
// A shape given on the command line (-DUCAP=... when the tuner builds its
// variants) takes precedence over the one recorded here.
#pragma once
#ifndef UCAP
#define UCAP 128
#endif
#ifndef LCAP
#define LCAP 16
#endif
#ifndef PU
#define PU 4
#endif
