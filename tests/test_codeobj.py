"""The gfx950 code objects inside the built library: every kernel keeps its
state in registers (no scratch memory) and reaches global memory through
global (not flat) instructions.  A kernel that spills, or whose arrays the
compiler demotes to the stack, loses most of its bandwidth without any change
in its results, so the parity tests cannot see it.  CPU only: the code objects
are unbundled from a copy of the library and read with the ROCm LLVM tools."""
import os
import re
import shutil
import subprocess

import pytest

b = pytest.importorskip("paper_1902_09931_amd.binding")

LLVM = "/opt/rocm/llvm/bin"


def _tool(name):
    path = os.path.join(LLVM, name)
    if not os.path.exists(path):
        pytest.skip(f"{path} not available")
    return path


@pytest.fixture(scope="module")
def code_objects(tmp_path_factory):
    objdump = _tool("llvm-objdump")
    d = tmp_path_factory.mktemp("cobj")
    lib = d / "lib.so"
    shutil.copy(b.library_path(), lib)
    subprocess.run([objdump, "--offloading", str(lib)], cwd=d, check=True,
                   stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    objs = sorted(p for p in d.iterdir() if p.name.endswith("gfx950"))
    assert objs, "no gfx950 code object in the library"
    return objs


def test_every_kernel_is_built_for_gfx950_without_scratch(code_objects):
    readelf = _tool("llvm-readelf")
    kernels = {}
    for obj in code_objects:
        notes = subprocess.run([readelf, "--notes", str(obj)], check=True,
                               capture_output=True, text=True).stdout
        name = None
        for line in notes.splitlines():
            m = re.match(r"\s+\.name:\s+(\S+)", line)
            if m:
                name = m.group(1)
            m = re.match(r"\s+\.private_segment_fixed_size:\s+(\d+)", line)
            if m and name is not None:
                kernels[name] = int(m.group(1))
                name = None
    # stencils, ragged 1D stencils, line solves, register line kernels, CH
    assert len(kernels) >= 150, len(kernels)
    spilled = {k: v for k, v in kernels.items() if v}
    assert not spilled, spilled


def test_no_flat_or_scratch_memory_instructions(code_objects):
    objdump = _tool("llvm-objdump")
    bad = re.compile(r"\b(flat|scratch)_(load|store|atomic)\w*")
    for obj in code_objects:
        asm = subprocess.run([objdump, "-d", str(obj)], check=True,
                             capture_output=True, text=True).stdout
        hits = bad.findall(asm)
        assert not hits, (obj.name, hits[:5])


def test_no_scalar_memory_writes(code_objects):
    """Global memory is written only through vector memory instructions: no
    scalar-cache store, atomic, write-back or discard appears in any kernel
    (kernels that write a table from one lane must still use vector stores)."""
    objdump = _tool("llvm-objdump")
    bad = re.compile(r"\bs_(store|buffer_store|atomic|buffer_atomic|dcache_wb|dcache_discard)\w*")
    for obj in code_objects:
        asm = subprocess.run([objdump, "-d", str(obj)], check=True,
                             capture_output=True, text=True).stdout
        hits = bad.findall(asm)
        assert not hits, (obj.name, hits[:5])
