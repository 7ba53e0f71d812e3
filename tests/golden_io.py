"""Reader for the worked-example fixtures under tests/golden/."""
import glob
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(path):
    rec = {"obs": {}, "tenv": {}}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, _, val = line.partition(":")
        val = val.strip()
        if key == "il":
            rec["il"] = val
        elif key == "tenv":
            rec["tenv"] = {k: int(v) for k, v in (kv.split("=") for kv in val.split())}
        elif key == "obs":
            for kv in val.split():
                lab_day, v = kv.split("=")
                lab, day = lab_day.split("@")
                rec["obs"][(lab, int(day))] = float(v)
        elif key == "discount_base":
            rec["disc"] = float(val)
        elif key == "parties":
            rec["parties"] = tuple(val.split())
        elif key == "expected":
            # a hand-derived arithmetic expression in numbers only
            rec["expected"] = float(eval(val, {"__builtins__": {}}, {}))
    return rec


def all_fixtures(prefix=""):
    return sorted(glob.glob(os.path.join(GOLDEN, prefix + "*.txt")))
