"""The boundary from plain C: include/dpd.h compiles as strict C99, a program
links against libdpd.so and the host-side checks answer without a device
(CPU only)."""
import os
import shutil
import subprocess

import pytest

from paper_1612_09001_amd import dpd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")
LIBDIR = os.path.dirname(dpd.LIB_PATH)

C_SRC = r"""
#include <stdio.h>
#include <string.h>

#include "dpd.h"

int main(void)
{
    const char *v = dpd_version();
    dpd_plan *p = NULL;
    int32_t even[1] = {2};
    int32_t odd[1] = {1};
    float c[4] = {1.f, 0.f, 0.f, 0.f};
    size_t bytes = 0;
    if (v == NULL || strstr(v, "gfx950") == NULL) return 1;
    /* even orders are rejected and the out-parameter stays untouched */
    if (dpd_create(even, 1, NULL, 0, 1, c, &p) == DPD_OK || p != NULL) return 2;
    if (dpd_create(odd, 1, NULL, 0, 0, c, &p) == DPD_OK || p != NULL) return 3;   /* L = 0 */
    if (dpd_apply(NULL, NULL, NULL, NULL, 16) != DPD_EINVAL) return 4;
    if (dpd_loss_ws_size(-1, &bytes) != DPD_EINVAL) return 5;
    if (dpd_ls_solve_ws_size(33, &bytes) != DPD_OK || bytes != 33u * 33u * 16u) return 6;
    if (strncmp(dpd_status_string(DPD_EINVAL), "DPD_", 4) != 0) return 7;
    printf("%s\n", v);
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_header_is_strict_c99_and_links(tmp_path):
    if not os.path.exists(dpd.LIB_PATH):
        pytest.skip("libdpd.so not built")
    src = tmp_path / "use_dpd.c"
    src.write_text(C_SRC)
    exe = tmp_path / "use_dpd"
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", INCLUDE, str(src), "-o", str(exe),
           "-L", LIBDIR, "-l:" + os.path.basename(dpd.LIB_PATH), "-Wl,-rpath," + LIBDIR,
           "-Wl,-rpath-link,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stderr)
    assert "gfx950" in r.stdout
