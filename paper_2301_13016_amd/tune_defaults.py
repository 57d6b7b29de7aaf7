"""Regenerate the built-in tuning table (csrc/pw_tune_defaults.inc) on the GPU.

Runs the library's autotuner (pw_tune) for the shape classes the library is
benchmarked and tested on and writes the chosen launch shapes as C
initialisers.  Rebuild the library afterwards.  Usage (on an MI355X):

    python paper_2301_13016_amd/tune_defaults.py [output.inc]
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

# (nx, ny, nz, dtype name, flags): forward for all storage types, adjoint and
# tangent for FP32/FP64, the z-fastest forward for the FP32 / FP64 classes
SHAPES = [
    (512, 512, 64, "float32", 15),
    (1024, 1024, 256, "float32", 9),
    (1024, 1024, 256, "bfloat16", 1),
    (1024, 1024, 256, "float16", 1),
    (256, 256, 128, "float32", 15),
    (64, 64, 64, "float64", 15),
    (16, 16, 16, "float64", 7),
    (128, 128, 128, "float32", 15),
    (256, 256, 256, "float32", 9),
    (512, 512, 128, "float32", 9),
    (1024, 1024, 256, "float64", 1),
    (512, 512, 64, "float64", 1),
]


def ceil_log2(x):
    return (int(x) - 1).bit_length()


def main(out_path):
    import torch
    from paper_2301_13016_amd import binding as B
    code = {"float32": B.PW_F32, "float64": B.PW_F64, "bfloat16": B.PW_BF16, "float16": B.PW_F16}
    tdt = {"float32": torch.float32, "float64": torch.float64, "bfloat16": torch.bfloat16, "float16": torch.float16}
    lines = ["// kind, dtype, log2 nx, log2 ny, log2 nz, cols/lane, rows/strip, z-chunks, waves/group, prefetch, "
             "share_rows",
             "// (kind 3, z-fastest: levels/lane, rows/strip, x-chunks, waves/group, prefetch, 0)",
             "// generated on %s by paper_2301_13016_amd/tune_defaults.py, unedited" % torch.cuda.get_device_name(0)]
    B.pw_tune_reset()
    for nx, ny, nz, dt, flags in SHAPES:
        B._check(B.pw_tune(B.pw_grid(nx, ny, nz, 1), code[dt], flags, None, None), "pw_tune")
        key = (ceil_log2(nx), ceil_log2(ny), ceil_log2(nz))
        for kind, name, bit, zext in ((0, "forward", 1, nz), (1, "adjoint", 2, nz + 2), (2, "tangent", 4, nz),
                                      (3, "zfast", 8, nx)):
            if not flags & bit:
                continue
            t = B.launch_shape(name, nx, ny, nz, tdt[dt])
            nzc = -(-zext // t[2])
            lines.append("{%d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d},  // %dx%dx%d %s %s" % (
                kind, code[dt], *key, t[0], t[1], nzc, t[3], t[4], t[5], nx, ny, nz, dt, name))
            print(lines[-1], flush=True)
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(HERE, "csrc", "pw_tune_defaults.inc"))
