"""The autotuner's search space and header (host side; the timing runs on
the GPU through `python -m paper_2609_05494_amd.autotune time`)."""
import re

from paper_2609_05494_amd import autotune


def test_space_holds_the_default_and_only_valid_shapes():
    assert autotune.DEFAULT in autotune.SPACE
    assert all(autotune.valid(s) for s in autotune.SPACE)
    assert len({autotune.tag(s) for s in autotune.SPACE}) == len(autotune.SPACE)
    assert not autotune.valid({"UCAP": 512, "LCAP": 16, "PU": 4})  # byte indices into a pass
    assert not autotune.valid({"UCAP": 192, "LCAP": 8, "PU": 8})   # a scan step overflows the list


def test_header_defines_the_winner(tmp_path):
    results = [{"shape": s, "ms_per_step": 1.0 + 0.01 * k, "digest": "x"} for k, s in enumerate(autotune.SPACE)]
    path = tmp_path / "wcsph_tuned.h"
    autotune.write_header(str(path), autotune.SPACE[3], "C4", 100, results, ["u1_l1_p1"])
    text = path.read_text()
    got = dict(re.findall(r"#define (\w+) (\d+)", text))
    assert got == {k: str(v) for k, v in autotune.SPACE[3].items()}
    assert "rejected" in text and text.count("//   ") == len(autotune.SPACE)
