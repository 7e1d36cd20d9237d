"""The autotuner's search space and header (host side; the timing runs on
the GPU through `python -m paper_2609_05494_amd.autotune time`)."""
import re

from paper_2609_05494_amd import autotune


def test_space_holds_the_default_and_only_valid_shapes():
    assert autotune.DEFAULT in autotune.SPACE
    assert all(autotune.valid(s) for s in autotune.SPACE)
    assert len({autotune.tag(s) for s in autotune.SPACE}) == len(autotune.SPACE)
    assert not autotune.valid({"UCAP": 512, "LCAP": 16, "RU": 2})  # byte indices into a pass
    assert not autotune.valid({"UCAP": 192, "LCAP": 4, "RU": 2})   # a list too short to hold a row's hits
    assert not autotune.valid({"UCAP": 192, "LCAP": 16, "RU": 3})


def test_header_defines_the_winner(tmp_path):
    results = [{"shape": s, "ms_per_step": 1.0 + 0.01 * k, "digest": "x"} for k, s in enumerate(autotune.SPACE)]
    path = tmp_path / "wcsph_tuned.h"
    autotune.write_header(str(path), autotune.SPACE[3], "C4", 100, results, ["u1_l1_r1"])
    text = path.read_text()
    got = dict(re.findall(r"#define (\w+) (\d+)", text))
    assert got == {k: str(v) for k, v in autotune.SPACE[3].items()}
    assert "rejected" in text and text.count("//   ") == len(autotune.SPACE)


def test_command_line_shape_wins_over_the_recorded_header():
    """A variant built with -DUCAP=... must get that shape, not the one the
    committed header records (the preprocessor output of the kernels file)."""
    import os
    import subprocess
    from paper_2609_05494_amd import build as hb
    src = os.path.join(hb.CSRC, "wcsph_kernels.hip")
    probe = "int ucap_probe = UCAP; int lcap_probe = LCAP; int ru_probe = RU;\n"
    text = open(src).read() + "\n" + probe
    cmd = [hb.hipcc(), "-x", "hip", "--offload-arch=gfx950", "--cuda-host-only", "-E", "-std=c++17",
           "-I", os.path.join(hb.ROOT, "include"), "-I", hb.CSRC, "-DUCAP=256", "-DRU=4", "-"]
    out = subprocess.run(cmd, input=text, capture_output=True, text=True, check=True).stdout
    got = dict(re.findall(r"int (\w+)_probe = (\d+);", out))
    assert got["ucap"] == "256" and got["ru"] == "4"
    assert got["lcap"] == re.search(r"#define LCAP (\d+)", open(autotune.HEADER).read()).group(1)
