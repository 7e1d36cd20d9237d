// Scan shapes of the pair pass, written by paper_2609_05494_amd/autotune.py.
// Workload C2, 1000 timed steps; ms per step of every shape:
//   u128_l16_r2: 0.0892
//   u128_l16_r4: 0.0904
//   u192_l16_r2: 0.0906
//   u128_l16_r1: 0.0907
//   u128_l24_r2: 0.0910
//   u192_l24_r2: 0.0919
//   u128_l24_r4: 0.0920
//   u192_l16_r4: 0.0920
//   u128_l24_r1: 0.0923
//   u192_l16_r1: 0.0925
//   u192_l24_r4: 0.0935
//   u192_l24_r1: 0.0939
//   u256_l16_r2: 0.0963
//   u256_l24_r2: 0.0963
//   u256_l24_r1: 0.0978
//   u256_l16_r1: 0.0978
//   u256_l16_r4: 0.0996
//   u256_l24_r4: 0.0996
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
