"""Host checks of the couplings' panel layout (csrc/batch.h), compiled with
hipcc as host code (no device needed):

  * jpanel_offset maps the n16 x ld padded couplings one to one onto
    [0, n16 * ld) for every element size, ragged n and several ld;
  * the step kernel's operand addresses (group base + chunk * group size *
    512 + panel-in-group * 512) equal jpanel_block for every aligned row
    tile of 1, 2, 4 and 8 panels and every chunk, clamped rows included.

The second check uses the helpers bstep_kernel forms its addresses with
(jpanel_group_base, jpanel_group_size) and the kernel's own clamping of
rows past n; a layout change that one side misses fails here, on the CPU,
before any GPU run.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2405_00366_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")

PROGRAM = r"""
#include <cstdio>
#include <vector>
#include "batch.h"
using namespace l0;
int main() {
  const int ns[] = {1, 15, 16, 17, 100, 127, 128, 129, 255, 300, 1203, 2000, 4096};
  for (int n : ns) {
    const int ld = (n + 31) / 32 * 32, np = (n + 15) / 16, nch = ld / 32;
    for (int esize : {1, 2, 4}) {
      std::vector<unsigned char> seen(size_t(np) * 16 * ld, 0);
      for (int r = 0; r < np * 16; ++r)
        for (int j = 0; j < ld; ++j) {
          const size_t o = jpanel_offset(r, j, ld, np, esize);
          if (o >= seen.size() || seen[o]) { printf("FAIL bijection n=%d esize=%d r=%d j=%d\n", n, esize, r, j); return 1; }
          seen[o] = 1;
        }
    }
    for (int RB : {1, 2, 4, 8}) {
      for (int p0 = 0; p0 < np; p0 += RB) {
        const int cstride = jpanel_group_size(p0, np) * 512;
        const size_t gbase = jpanel_group_base(p0, nch);
        for (int rb = 0; rb < RB; ++rb) {
          const int pp = (p0 + rb) * 16 < n ? p0 + rb : p0;
          for (int c = 0; c < nch; ++c) {
            const size_t a = gbase + size_t(c * cstride) + (pp % kPanelGroup) * 512;
            if (a != jpanel_block(pp, c, nch, np)) { printf("FAIL tile n=%d RB=%d p0=%d rb=%d c=%d\n", n, RB, p0, rb, c); return 1; }
          }
        }
      }
    }
  }
  printf("OK\n");
  return 0;
}
"""


def _hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_panel_layout_bijective_and_matches_tile_addressing(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not found")
    src = tmp_path / "layout.hip"
    src.write_text(PROGRAM)
    exe = tmp_path / "layout"
    cmd = [hipcc, "-O1", "-std=c++17", "--offload-arch=gfx950", f"-I{INCLUDE}", f"-I{CSRC}", str(src), "-o", str(exe)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stdout + res.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "OK", out.stdout + out.stderr
