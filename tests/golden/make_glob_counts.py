"""Writes glob_counts.json from the closed-form counts of box partitions (no solver code)."""
import json
import os


def counts(S):
    V = S * (S + 1) ** 2 - 4
    E = S * ((S + 1) ** 2 - 4) + 2 * S * (S * (S + 1) - 2)
    F = 3 * (S - 1) * S * S
    return {"V": V, "E": E, "F": F, "coarse_V": 3 * V, "coarse_VE": 3 * (V + E),
            "coarse_VEF": 3 * (V + E + F)}


if __name__ == "__main__":
    out = {str(S): counts(S) for S in (2, 3, 4, 8)}
    with open(os.path.join(os.path.dirname(__file__), "glob_counts.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
