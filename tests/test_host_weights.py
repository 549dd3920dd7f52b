"""Host logic of the library, compiled with g++ (no GPU): the acoustic
stencils in mirror-orbit form against the dense stencils they regroup."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2205_07572_amd", "csrc")


def test_orbit_weights_regroup_the_dense_stencils(tmp_path):
    exe = str(tmp_path / "host_weights_check")
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-D__host__=", "-D__device__=", f"-I{CSRC}",
                           f"-I{os.path.join(ROOT, 'include')}", "-o", exe,
                           os.path.join(ROOT, "tests", "host_weights_check.cpp"), os.path.join(CSRC, "af_weights.cpp")])
    r = subprocess.run([exe], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
