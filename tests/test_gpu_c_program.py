"""GPU test: a plain C program (tests/native/c_abi_roundtrip.c) drives the library through
include/ckks_mi355x.h alone -- keys, plain and value-cached encryption, the 3x3 mean
filter, decryption, an error path -- and checks the decrypted pixels."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_c_program_roundtrip(tmp_path):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib_dir = os.path.join(ROOT, "paper_2409_03568_amd")
    exe = str(tmp_path / "c_abi_roundtrip")
    subprocess.run(["gcc", "-std=c99", "-O1", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", "-o", exe, os.path.join(HERE, "native", "c_abi_roundtrip.c"),
                    "-L", lib_dir, "-lckks_mi355x", "-L", "/opt/rocm/lib", "-lamdhip64", "-lm",
                    "-Wl,-rpath," + lib_dir + ":/opt/rocm/lib"], check=True, capture_output=True)
    print("[gpu] C program through the ABI", flush=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip() == "OK"
