"""The values the paper prints (tests/golden/printed_values.txt) as a dict name -> float."""
import os

_HERE = os.path.dirname(os.path.abspath(__file__))


def printed() -> dict:
    out = {}
    with open(os.path.join(_HERE, "printed_values.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                name, value = (s.strip() for s in line.split("=", 1))
                out[name] = float(value)
    return out
