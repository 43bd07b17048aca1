"""CPU checks of the C ABI: the built library loads and exports every entry
point that include/msrsb.h declares, and the binding declares the same set.
No compute call is made (there may be no GPU)."""
import ctypes
import os
import re
import subprocess


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msrsb.h")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(msrsb_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_paper_calls():
    names = declared_symbols()
    for must in ["msrsb_set_matrix", "msrsb_set_coarse", "msrsb_setup_basis",
                 "msrsb_build_coarse", "msrsb_apply_preconditioner", "msrsb_solve",
                 "msrsb_solve_transpose", "msrsb_tpfa_adjoint_grad", "msrsb_assemble_tpfa",
                 "msrsb_assemble_q1", "msrsb_q1_adjoint_grad"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1912_06934_amd import _binding
    lib = _binding.load()
    out = subprocess.run(["nm", "-D", "--defined-only", _binding.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (msrsb_[a-z0-9_]+)", out))
    missing = [s for s in declared_symbols() if s not in exported]
    assert not missing, missing
    for s in declared_symbols():
        assert isinstance(getattr(lib, s), ctypes._CFuncPtr)


def test_binding_covers_the_header():
    from paper_1912_06934_amd import _binding
    bound = sorted(name for name, _, _ in _binding.SIGNATURES)
    assert bound == declared_symbols()


def test_library_is_built_for_gfx950():
    from paper_1912_06934_amd import _binding
    blob = open(_binding.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


def test_oracle_and_library_share_no_source():
    lib_dir = os.path.join(ROOT, "paper_1912_06934_amd")
    for dirpath, _, files in os.walk(lib_dir):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt
                assert "oracle.c" not in txt
    otxt = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    assert "#include \"internal.h\"" not in otxt and "msrsb.h" not in otxt
