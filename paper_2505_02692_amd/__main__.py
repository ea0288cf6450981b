"""Command line: the ZeroSpeech phoneme / triphone ABX error rate.

    python -m paper_2505_02692_amd ITEM_FILE FEATURES_DIR --frame-step 0.02
        [--speaker within|across] [--context within|any]
        [--distance angular|euclidean] [--mode dtw|pooled] [--libri-light]

FEATURES_DIR holds one file per utterance named in the item file:
<name>.npy ([n_frames, dim] float32, loaded without pickle) or <name>.pt (a
tensor, loaded with weights_only=True).  Prints one JSON line.
"""
import argparse
import json
import os
import sys


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m paper_2505_02692_amd", description=__doc__.splitlines()[0])
    ap.add_argument("item_file")
    ap.add_argument("features_dir")
    ap.add_argument("--frame-step", type=float, required=True, help="seconds between feature frames")
    ap.add_argument("--speaker", choices=("within", "across"), default="within")
    ap.add_argument("--context", choices=("within", "any"), default="within")
    ap.add_argument("--distance", choices=("angular", "euclidean"), default="angular")
    ap.add_argument("--mode", choices=("dtw", "pooled"), default="dtw")
    ap.add_argument("--libri-light", action="store_true", help="the Libri-Light slicing (one frame fewer)")
    ap.add_argument("--device", type=int, default=0)
    args = ap.parse_args(argv)

    import numpy as np
    import torch
    from . import Context, read_item_file, zerospeech_abx

    _, files, _, _, _ = read_item_file(args.item_file)
    feats = {}
    for name in sorted(set(files)):
        npy = os.path.join(args.features_dir, name + ".npy")
        pt = os.path.join(args.features_dir, name + ".pt")
        if os.path.exists(npy):
            x = torch.from_numpy(np.load(npy, allow_pickle=False).astype(np.float32, copy=False))
        elif os.path.exists(pt):
            x = torch.load(pt, map_location="cpu", weights_only=True)
        else:
            print(f"no features for {name!r} in {args.features_dir}", file=sys.stderr)
            return 2
        feats[name] = x.contiguous().to(f"cuda:{args.device}")
    torch.cuda.set_device(args.device)
    err = zerospeech_abx(Context(args.device), args.item_file, feats, args.frame_step, args.speaker,
                         args.context, args.distance, args.mode, libri_light=args.libri_light)
    print(json.dumps({"abx_error": err, "speaker": args.speaker, "context": args.context,
                      "distance": args.distance, "mode": args.mode, "libri_light": args.libri_light}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
