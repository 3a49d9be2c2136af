"""libjt.so and torch must share one HIP runtime (no GPU involved).

torch's libtorch_hip.so asks for the unversioned name libamdhip64.so and
finds its own copy through its RPATH, while libjt.so asks for the soname
libamdhip64.so.7.  Loaded after torch, libjt.so's request is met by the
runtime torch already mapped (same soname); loaded before torch, the two
requests resolve to two different files and the process ends up with two HIP
and two HSA runtimes, with torch's device pointers launched on the other
runtime's queues.  The binding imports torch first and refuses to load when
two runtimes are mapped.  These checks run in child processes so that the
test session's own imports do not matter.
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MAPS = ("sorted({l.split()[-1] for l in open('/proc/self/maps') "
        "if 'libamdhip64' in l or 'libhsa-runtime64' in l})")


def _run(code):
    env = dict(os.environ, PYTHONPATH=ROOT)
    return subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=ROOT,
                          timeout=300)


def test_binding_maps_one_hip_runtime():
    r = _run("import paper_1901_07275_amd; print(len(%s))" % MAPS)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().splitlines()[-1] == "2"  # one libamdhip64 and one libhsa-runtime64


def test_loading_the_library_before_torch_maps_two_runtimes_and_the_binding_refuses():
    code = ("import ctypes, paper_1901_07275_amd.build as b, os\n"
            "ctypes.CDLL(os.path.join(os.path.dirname(b.__file__), 'libjt.so'))\n"
            "try:\n"
            "    import paper_1901_07275_amd\n"
            "    print('imported')\n"
            "except ImportError as e:\n"
            "    print('refused:', e)\n"
            "print(len(%s))\n" % MAPS)
    # import the build module by path: importing it as a submodule would run the
    # package's __init__ (and import torch) first
    code = code.replace("import ctypes, paper_1901_07275_amd.build as b, os",
                        "import ctypes, os, importlib.util as u\n"
                        "s = u.spec_from_file_location('b', 'paper_1901_07275_amd/build.py')\n"
                        "b = u.module_from_spec(s); s.loader.exec_module(b)")
    r = _run(code)
    assert r.returncode == 0, r.stderr
    lines = r.stdout.strip().splitlines()
    assert lines[0].startswith("refused:"), lines
    assert lines[-1] == "4"  # two HIP and two HSA runtimes
