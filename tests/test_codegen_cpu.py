"""The generated fused-broadcast header matches its generator, and its asm
follows the scheme the generator documents."""
import os
import re
import subprocess
import sys

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2608_25469_amd", "csrc")


def test_dpp_fma_header_is_current():
    out = subprocess.run([sys.executable, os.path.join(CSRC, "gen_dpp_fma.py")], capture_output=True,
                         text=True, check=True).stdout
    with open(os.path.join(CSRC, "dpp_fma.h")) as f:
        assert f.read() == out


def test_dpp_fma_rows_and_order():
    with open(os.path.join(CSRC, "dpp_fma.h")) as f:
        text = f.read()
    bodies = re.findall(r"fnma_rows<(false|true), (\d+)>\(.*?\{\n    asm volatile\((.*?)\n        :", text, re.S)
    assert len(bodies) == 32
    for cx, i0, body in bodies:
        i0 = int(i0)
        ins = re.findall(r'"([^"]*)\\n"', body)
        assert ins[0] == "s_nop 1"
        rows = [int(m) for m in re.findall(r"row_newbcast:(\d+)", body)]
        per = 4 if cx == "true" else 1
        # every row of [i0, 16) once (four times for complex), ascending
        assert rows == [r for r in range(i0, 16) for _ in range(per)]
        if cx == "true":
            n = 16 - i0
            cr, ci, xr, xi = 2 * n, 2 * n + 1, 2 * n + 2, 2 * n + 3
            for j in range(n):
                quad = ins[1 + 4 * j: 5 + 4 * j]
                # yr -= lr xr, yi -= lr xi, yr += li xi, yi -= li xr
                assert quad[0].startswith(f"v_fmac_f64_dpp %{j}, -%{cr}, %{xr} ")
                assert quad[1].startswith(f"v_fmac_f64_dpp %{n + j}, -%{cr}, %{xi} ")
                assert quad[2].startswith(f"v_fmac_f64_dpp %{j}, %{ci}, %{xi} ")
                assert quad[3].startswith(f"v_fmac_f64_dpp %{n + j}, -%{ci}, %{xr} ")
        else:
            n = 16 - i0
            for j in range(n):
                assert ins[1 + j].startswith(f"v_fmac_f64_dpp %{j}, -%{n}, %{n + 1} ")
