"""Host-side checks of device helpers that need no GPU: the look-back flag
word of the cell-list sort (epoch tag, status, value) across the wrap of its
30-bit epoch field. The helpers are compiled from the library's own header
into a host program with hipcc and run on the CPU."""
import os
import subprocess

import pytest

from paper_2609_05494_amd import build as hb

PROG = r"""
#include "wcsph_dev.h"
#include <cstdio>
int main() {
  const uint32_t starts[] = {1u, (1u << 30) - 3u, (1u << 31) + 5u, 0xfffffffcu};
  int bad = 0;
  for (uint32_t s0 : starts)
    for (uint32_t k = 0; k < 8; ++k) {
      const uint32_t e = s0 + k;  // the epoch counter of consecutive sorts (wraps at 2^32)
      for (uint32_t status = 1; status <= 2; ++status) {
        const unsigned long long f = tile_word(e, status, 0xdeadbeefu);
        bad += !tile_epoch_is(f, e);                      // a flag of this sort matches
        bad += tile_epoch_is(f, e + 1u);                  // and is stale for the next one
        bad += tile_epoch_is(tile_word(e - 1u, status, 7u), e);  // the previous sort's flag
        bad += (uint32_t)f != 0xdeadbeefu || ((uint32_t)(f >> 32) & 3u) != status;
      }
    }
  std::printf("bad=%d\n", bad);
  return bad != 0;
}
"""


def test_sort_flag_epoch_survives_the_30_bit_wrap(tmp_path):
    src = tmp_path / "flags.hip"
    src.write_text(PROG)
    exe = tmp_path / "flags"
    cmd = [hb.hipcc(), "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17", "-I", hb.CSRC,
           "-I", os.path.join(hb.ROOT, "include"), str(src), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail(r.stderr[-2000:])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "bad=0" in out.stdout
