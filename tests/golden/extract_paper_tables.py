"""Write paper_tables.json from the LaTeX source of the paper's tables (run once, by hand,
where the paper's text is available; the tests read only the JSON).

Extracted mechanically, so the numbers typed into workloads.py are checked against an
independent route: the true-parameter tables of App. B (spectral_true_params,
spectral_true_K3, spectral_true_K10, spectral_true_K30) and App. E (xrd_true_phase,
xrd_true_bg), the prior tables spectral_priors and xrd_priors (constant entries), and the
heteroscedastic noise parameters of App. D.

Usage: python tests/golden/extract_paper_tables.py <file holding the LaTeX source of the
paper's App. B, D and E tables>
"""
import json
import os
import re
import sys


def table_rows(src, label):
    i = src.index(r"\label{tab:" + label + "}")
    body = src[src.index(r"\begin{tabular}", i):src.index(r"\end{tabular}", i)]
    body = body.split(r"\hline", 1)[1]
    rows = []
    for line in body.split(r"\\"):
        line = line.strip()
        if not line or line.startswith(r"\hline") or line.startswith(r"\multicolumn"):
            continue
        rows.append([c.strip() for c in line.replace(r"\hline", "").split("&")])
    return rows


def num(cell):
    return float(re.sub(r"[{}\\,]", "", cell))


def prior(cell):
    """Ga(a, b) / N(m, v) / U(a, b) with numeric arguments, else None."""
    m = re.match(r"\$\\mathrm\{Ga\}\(([-\d.]+),\s*([-\d.]+)\)\$", cell)
    if m:
        return ["gamma", float(m.group(1)), float(m.group(2))]
    m = re.match(r"\$\\mathcal\{N\}\(([-\d.]+),\s*([-\d.]+)(\^2)?\)\$", cell)
    if m:
        return ["normal_var", float(m.group(1)), float(m.group(2)) ** (2 if m.group(3) else 1)]
    m = re.match(r"\$\\mathrm\{U\}\(([-\d.]+),\s*([-\d.]+)\)\$", cell)
    if m:
        return ["uniform", float(m.group(1)), float(m.group(2))]
    return None


def main(path):
    src = open(path).read()
    out = {"_source": "arXiv 2604.03271, App. B, D and E tables (label named per entry)"}
    out["spectral_true_params"] = {str(int(num(r[0]))): [int(num(r[1])), r[2], num(r[3])]
                                   for r in table_rows(src, "spectral_true_params")}
    for K in (3, 10, 30):
        out[f"spectral_true_K{K}"] = [[num(c) for c in r[1:]] for r in table_rows(src, f"spectral_true_K{K}")]
    sp = table_rows(src, "spectral_priors")
    out["spectral_priors"] = {K: [prior(r[2 + j]) for r in sp] for j, K in enumerate(("3", "10", "30"))}
    out["xrd_true_phase"] = {r[0]: [num(c) for c in r[1:]] for r in table_rows(src, "xrd_true_phase")}
    out["xrd_true_phase_columns"] = ["A", "shift", "alpha", "r", "u", "v", "w", "s", "t"]
    out["xrd_true_bg"] = [num(c) for c in table_rows(src, "xrd_true_bg")[0]]
    out["xrd_priors"] = {re.sub(r"[$\\{}]", "", r[0]).strip(): prior(r[2]) for r in table_rows(src, "xrd_priors")}
    m = re.search(r"\\sigma_0\{=\}([\d.]+).*?\\sigma_1\{=\}([\d.]+).*?\\sigma_2\{=\}([\d.]+)", src, re.S)
    out["xps_noise"] = [float(m.group(i)) for i in (1, 2, 3)]
    dst = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_tables.json")
    json.dump(out, open(dst, "w"), indent=1)
    print("wrote", dst)


if __name__ == "__main__":
    main(sys.argv[1])
