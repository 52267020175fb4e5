"""The per-edge support word (csrc/common.h) on the host: the library's own helpers,
compiled by hipcc into a small host program, against the layout they promise --
support in the upper 29 bits (two's complement), edge state in the low 3 bits, a
decrement that never touches the state, a tag joined by OR and retired by XOR, and
the three rotating round tags of the sub-level loop (PKT section, Algorithm 4's
inCurr / inNext / processed flags)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1707_02000_amd", "csrc")

PROGRAM = r"""
#include "common.h"
#include <stdio.h>
int main() {
  const int sups[] = {-(1 << 28), -100000, -2, -1, 0, 1, 2, 7, 8, 9, 1000, SW_MAX_SUPPORT - 1, SW_MAX_SUPPORT};
  int bad = 0;
  for (int s : sups)
    for (int st = 0; st < 5; ++st) {
      const int w = sw_make(s, (u8)st);
      if (sw_sup(w) != s || sw_st(w) != st) ++bad;
      if (s > -(1 << 28)) {  // a decrement leaves the state alone, also below zero
        const int d = w - SW_ONE;
        if (sw_sup(d) != s - 1 || sw_st(d) != st) ++bad;
      }
      if (s < SW_MAX_SUPPORT) {  // and so does the undo
        const int u = w + SW_ONE;
        if (sw_sup(u) != s + 1 || sw_st(u) != st) ++bad;
      }
    }
  for (int r = 0; r < 9; ++r) {
    const u8 t = round_tag(r);
    if (t < 2 || t > 4) ++bad;
    if (t == round_tag(r + 1) || t == round_tag(r + 2) || round_tag(r + 1) == round_tag(r + 2)) ++bad;
    if (t != round_tag(r + 3)) ++bad;
    // alive at support 5 joins the next frontier by OR, then retires by XOR
    const int joined = sw_make(5, ST_ALIVE) | (int)round_tag(r + 1);
    if (sw_st(joined) != round_tag(r + 1) || sw_sup(joined) != 5) ++bad;
    const int retired = joined ^ (int)(round_tag(r + 1) ^ ST_PROC);
    if (sw_st(retired) != ST_PROC || sw_sup(retired) != 5) ++bad;
    // during round r: current = tag(r), next = tag(r + 1), processed = PROC or tag(r - 1)
    if (is_processed(round_tag(r), r) || is_processed(round_tag(r + 1), r) || is_processed(ST_ALIVE, r)) ++bad;
    if (!is_processed(ST_PROC, r) || !is_processed(round_tag(r + 2), r)) ++bad;
    if (r > 0 && !is_processed(round_tag(r - 1), r)) ++bad;
  }
  printf("bad %d\n", bad);
  return bad != 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not on PATH")
def test_support_word_layout(tmp_path):
    src = tmp_path / "sw_check.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "sw_check"
    subprocess.run(["hipcc", "-x", "hip", "--offload-arch=gfx950", "-O1", "-I", CSRC, str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip() == "bad 0"
