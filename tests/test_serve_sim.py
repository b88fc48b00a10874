"""The serving loop's bookkeeping (admission by budget, slots and pool
regions, retirement, cancellation, tick pipelining) on a fake device, on the
CPU: hb_serve.cpp is compiled with g++ against tests/serve_sim/fake_device.cpp,
which backs the HIP calls with host memory, converges every graph after a
known number of passes and checks the row-list and region invariants the
real kernels rely on at every pass."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SIM = os.path.join(ROOT, "tests", "serve_sim")


def _build(out, extra=()):
    subprocess.check_call(
        ["g++", "-std=c++17", "-O1", "-g", *extra, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
         "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_1308_2144_amd", "csrc"),
         "-pthread", os.path.join(SIM, "drive.cpp"), os.path.join(SIM, "fake_device.cpp"),
         os.path.join(ROOT, "paper_1308_2144_amd", "csrc", "hb_serve.cpp"), "-o", out])
    return out


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    return _build(str(tmp_path_factory.mktemp("serve_sim") / "drive"))


@pytest.fixture(scope="module")
def sim_checked(tmp_path_factory):
    """The same loop built with the address and undefined-behaviour checkers
    (host code only: the device is the fake one)."""
    return _build(str(tmp_path_factory.mktemp("serve_sim_checked") / "drive"),
                  ("-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"))


@pytest.mark.parametrize("args", [["list"], ["list", "tight"], ["stress", "1"], ["stress", "2"],
                                  ["stress", "3"], ["stress", "7"]])
def test_serving_loop_on_fake_device(sim, args):
    p = subprocess.run([sim, *args], capture_output=True, text=True, timeout=240)
    assert p.returncode == 0 and p.stdout.strip().endswith("ok"), p.stdout[-2000:] + p.stderr[-4000:]


@pytest.mark.parametrize("args", [["list"], ["list", "tight"], ["stress", "1"], ["stress", "7"]])
def test_serving_loop_under_address_and_ub_checkers(sim_checked, args):
    p = subprocess.run([sim_checked, *args], capture_output=True, text=True, timeout=240)
    assert p.returncode == 0 and p.stdout.strip().endswith("ok"), p.stdout[-2000:] + p.stderr[-4000:]
