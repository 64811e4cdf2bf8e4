"""Parser for the paper's worked example (paper_example.txt)."""
import os

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_example.txt")


def load(path: str = PATH) -> dict:
    d = {"search": {}, "occ": {}, "row": {}}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, *vals = line.split()
        if key == "text":
            d["text"] = vals[0]
        elif key == "search":
            d["search"][vals[0]] = (int(vals[1]), int(vals[2]))
        elif key == "occ":
            d["occ"][vals[0]] = [int(v) for v in vals[1:]]
        elif key == "row":
            d["row"][int(vals[0])] = vals[1]
        elif key == "rank_sample":
            d[key] = [None if v == "-" else int(v) for v in vals]
        else:
            d[key] = [int(v) for v in vals]
    return d
