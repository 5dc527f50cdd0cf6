"""Measured device rates of one MI355X next to the datasheet peaks the roofline
fractions use: FP64 / FP32 / BF16 matrix-core loops and a device copy
(flame_probe).  Prints a markdown table.

    python -m paper_1601_05871_amd.peaks [--copy-gib 2]
"""
from __future__ import annotations

import argparse

DATASHEET = {"mfma_f64": (78.6, "TFLOP/s"), "mfma_f32": (157.3, "TFLOP/s"), "mfma_bf16": (2500.0, "TFLOP/s"),
             "copy": (8000.0, "GB/s")}
WORK = {"mfma_f64": 2000, "mfma_f32": 2000, "mfma_bf16": 2000}  # rounds of 16 x 4 instructions


def main() -> None:
    import torch

    import paper_1601_05871_amd as fl

    ap = argparse.ArgumentParser()
    ap.add_argument("--copy-gib", type=float, default=2.0)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    props = torch.cuda.get_device_properties(dev)
    sink = torch.empty(props.multi_processor_count * 8 * 256, dtype=torch.float32, device=dev)
    print(f"device: {props.name}, {props.multi_processor_count} CUs")
    print("| probe | workgroups per CU (4 wavefronts each) | measured | datasheet | fraction |\n"
          "|---|---|---|---|---|")
    for kind in ("mfma_f64", "mfma_f32", "mfma_bf16"):
        peak, unit = DATASHEET[kind]
        for wg in (1, 2, 4, 8):
            r = fl.probe(kind, WORK[kind], sink, args.reps, wg_per_cu=wg)
            print(f"| {kind} | {wg} | {r:.1f} {unit} | {peak} {unit} | {r / peak:.3f} |", flush=True)
    nbytes = int(args.copy_gib * (1 << 30)) // 16 * 16
    buf = torch.empty(2 * nbytes, dtype=torch.uint8, device=dev)
    r = fl.probe("copy", nbytes, buf, args.reps)
    peak, unit = DATASHEET["copy"]
    print(f"| copy ({args.copy_gib:g} GiB, read + write) | 2 | {r:.0f} {unit} | {peak:.0f} {unit} | {r / peak:.3f} |")


if __name__ == "__main__":
    main()
