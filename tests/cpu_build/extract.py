"""Extract the kernel sections of the library sources into host-compilable
include files for the threaded CPU build (the launch sections, which use the
triple-chevron syntax, are left out; harness.cpp provides CPU launchers).

Usage: python extract.py OUTDIR
"""
import os
import shutil
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(ROOT, "paper_1501_07844_amd", "csrc")


def cut(text, start_marker, end_marker):
    i = text.index(start_marker)
    return text[i:text.index(end_marker, i)]


def main(out):
    os.makedirs(out, exist_ok=True)
    # the empty asm that hides a value from the optimiser names a VGPR operand
    k = open(os.path.join(SRC, "pf_kernels.hip")).read().replace(
        '__asm__ volatile("" : "+v"(v));', '__asm__ volatile("" : "+r"(v));')
    kd = k
    k = k[:k.index("// ----------------------------------------------------------- dispatch ----")]
    k += "\n}  // namespace\n" + cut(kd, "bool lds_supported(", "hipError_t launch_lds(")
    k += cut(kd, "bool tile_supported(", "hipError_t launch_tile(")
    k += "\n}  // namespace pf\n"
    f = open(os.path.join(SRC, "pf_fused.hip")).read()
    fk = f[:f.index("template <int ND, typename T, typename F>\nhipError_t fused_bucket")]
    fk += "\n}  // namespace\n" + cut(f, "bool fused_supported(", "hipError_t launch_fused(")
    fk += "\n}  // namespace pf\n"
    fl = open(os.path.join(SRC, "pf_flowlabel.hip")).read().replace(
        '__asm__ volatile("" : "+s"(v));', '__asm__ volatile("" : "+r"(v));')
    flk = fl[:fl.index("// ----------------------------------------------------------- dispatch ----")]
    flk += "\n}  // namespace\n" + cut(fl, "bool flow_label_supported(", "hipError_t launch_flow_label(")
    flk += "\n}  // namespace pf\n"
    a = open(os.path.join(SRC, "pf_adjoint.hip")).read()
    ak = a[:a.index("unsigned sblocks(size_t n)")] + "\n}  // namespace\n"
    ak += cut(a, "bool adj_fused_supported(", "hipError_t launch_adj_flow(") + "\n}  // namespace pf\n"
    ff = open(os.path.join(SRC, "pf_fullflow.hip")).read()
    ffk = ff[:ff.index("template <typename F>\nhipError_t ff_dispatch")] + "\n}  // namespace\n"
    ffk += cut(ff, "bool ff_supported(", "hipError_t launch_ff_init(") + "\n}  // namespace pf\n"
    # the constant address space cast has no host meaning
    d = open(os.path.join(SRC, "pf_device.h")).read().replace(
        "using cfloat = const __attribute__((address_space(4))) float;", "using cfloat = const float;")
    for name, text in (("kernels.inc", k), ("fused.inc", fk), ("flowlabel.inc", flk), ("adjoint.inc", ak),
                       ("fullflow.inc", ffk), ("pf_device.h", d)):
        with open(os.path.join(out, name), "w") as fh:
            fh.write(text)
    for name in ("pf_api.cpp", "pf_internal.h", "pf_fullflow.h"):
        shutil.copy(os.path.join(SRC, name), os.path.join(out, name))
    shutil.copy(os.path.join(ROOT, "include", "pseudoflow.h"), os.path.join(out, "pseudoflow.h"))


if __name__ == "__main__":
    main(sys.argv[1])
