"""The block coder of compressed streamed graphs (host code,
paper_1308_2144_amd/csrc/hb_stream_codes.h) on the CPU: tests/stream_codes/
check.cpp codes random sorted rows and extreme id sequences and reads them
back with a decoder written from the format's description, under the address
and undefined-behaviour checkers (the device decoder is checked by the
streamed GPU tests)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_block_coder_round_trip(tmp_path):
    exe = str(tmp_path / "check")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined",
                           "-I" + os.path.join(ROOT, "paper_1308_2144_amd", "csrc"),
                           os.path.join(ROOT, "tests", "stream_codes", "check.cpp"), "-o", exe])
    p = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert p.returncode == 0 and p.stdout.strip().endswith("ok"), p.stdout[-2000:] + p.stderr[-4000:]
