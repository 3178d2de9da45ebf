"""Concurrent context set-up is race-free (CPU, host code only).

The library's element constants are built on the host by every hmg_create and
hmg_batch_create.  This test builds that host code with ThreadSanitizer (host
side only; no device code is instrumented), runs it from 16 threads at once
and requires no reported race and identical results in every thread.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2301_08911_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

DRIVER = r"""
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>
#include "hmg_internal.hpp"
int main() {
  static hmg::ElementConsts ref, out[16];
  char err[256];
  if (hmg::build_element_consts(0.3, &ref, err, sizeof(err))) { std::printf("%s\n", err); return 2; }
  std::vector<std::thread> th;
  for (int t = 0; t < 16; ++t)
    th.emplace_back([t] {
      char e[256];
      for (int r = 0; r < 20; ++r) hmg::build_element_consts(0.3, &out[t], e, sizeof(e));
    });
  for (auto& x : th) x.join();
  for (int t = 0; t < 16; ++t)
    if (std::memcmp(&out[t], &ref, sizeof(ref))) { std::printf("thread %d differs\n", t); return 3; }
  std::printf("ok\n");
  return 0;
}
"""


@pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which("hipcc")), reason="no hipcc")
def test_element_constants_are_race_free_across_threads(tmp_path):
    src = tmp_path / "driver.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    build = [HIPCC, "-O1", "-g", "-std=c++17", "-Xarch_host", "-fsanitize=thread",
             "-fno-gpu-sanitize", "-I", CSRC, str(src), os.path.join(CSRC, "element.cpp"),
             "-o", str(exe), "-pthread"]
    res = subprocess.run(build, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stderr[-3000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert res.returncode == 0, (res.returncode, res.stdout[-2000:], res.stderr[-3000:])
    assert res.stdout.strip() == "ok"
    assert "ThreadSanitizer" not in res.stderr
