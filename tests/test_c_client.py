"""The C ABI from a plain C client: include/kbuild.h compiles as C99 (gcc, warnings as
errors), the program links against libkbuild.so and calls the host-only entry points
(version, status strings, workspace planning for every build kind, argument errors).
No GPU is touched: kb_plan* read only sizes."""
from __future__ import annotations

import os
import subprocess

import pytest

from paper_1501_04784_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROGRAM = r"""
#include <stdio.h>
#include <string.h>
#include "kbuild.h"

#define CHECK(c) do { if (!(c)) { printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c); return 1; } } while (0)

int main(void) {
  size_t ws = 0, ws_dof = 0, ws_grp = 0, ws_adj = 0, ws_bat = 0;
  int64_t nt = 0, nt_dof = 0;
  kb_mesh m;
  kb_batch b;
  kb_tuning tu;
  memset(&m, 0, sizeof m);
  memset(&b, 0, sizeof b);
  memset(&tu, 0, sizeof tu);
  CHECK(kb_version() == KB_VERSION);
  CHECK(strcmp(kb_status_string(KB_OK), "ok") == 0);
  CHECK(strcmp(kb_status_string(KB_ENOSPC), "workspace too small") == 0);

  m.elem = KB_TET4; m.op = KB_OP_STIFFNESS; m.n_elem = 6000; m.n_node = 1331;
  CHECK(kb_plan(&m, KB_FP32_FB64, NULL, &ws, &nt) == KB_OK);
  CHECK(nt == 6000 * 10 && ws > 0);
  CHECK(kb_plan(&m, KB_FP32_FB64, &tu, NULL, NULL) == KB_OK);
  CHECK(kb_plan_dof(&m, 3, KB_FP64, NULL, &ws_dof, &nt_dof) == KB_OK);
  CHECK(nt_dof == 6000 * 78 && ws_dof > ws);
  CHECK(kb_plan_grouped(&m, KB_FP32, NULL, 1000, 20000, &ws_grp) == KB_OK && ws_grp > 0);
  CHECK(kb_plan_adjoint(&m, &ws_adj) == KB_OK && ws_adj > 0);
  b.elem = KB_HEX8; b.n_mesh = 3; b.n_elem = 300; b.n_node = 500;
  CHECK(kb_plan_batched(&b, KB_FP64, NULL, &ws_bat, NULL) == KB_OK && ws_bat > 0);

  /* argument errors come back before anything is enqueued */
  CHECK(kb_plan(NULL, KB_FP64, NULL, &ws, NULL) == KB_EINVAL);
  m.elem = 5;
  CHECK(kb_plan(&m, KB_FP64, NULL, &ws, NULL) == KB_EINVAL);
  m.elem = KB_HEX8;
  CHECK(kb_plan(&m, 7, NULL, &ws, NULL) == KB_EINVAL);
  CHECK(kb_plan_dof(&m, 4, KB_FP64, NULL, &ws, NULL) == KB_EINVAL);
  CHECK(kb_plan_grouped(&m, KB_FP64, NULL, 0, 10, &ws) == KB_EINVAL);
  CHECK(kb_build_lower_csr(&m, KB_FP64, NULL, NULL, 0, NULL, NULL, NULL, 0, NULL, NULL, NULL) == KB_EINVAL);
  printf("ok %zu %zu %zu %zu %zu\n", ws_dof, ws_grp, ws_adj, ws_bat, (size_t)nt_dof);
  return 0;
}
"""


def test_c99_client_compiles_links_and_plans(tmp_path):
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    src = tmp_path / "client.c"
    src.write_text(PROGRAM)
    exe = tmp_path / "client"
    libdir = os.path.dirname(_lib.LIB_PATH)
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
           str(src), "-o", str(exe), os.path.abspath(_lib.LIB_PATH), f"-Wl,-rpath,{libdir}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert run.returncode == 0, run.stdout + run.stderr
    assert run.stdout.startswith("ok ")
