"""Write the paper's printed coefficient and convergence tables as text fixtures.

Reads the LaTeX source of the paper (H. Shen, arXiv 2311.15504), whose path
is the one command-line argument, and writes, next to this script:

* a_coefficients.txt  - Tables Flux_reconstruction1/2 (a_l, Sec. 3.1)
* b_coefficients.txt  - Tables ISCoe1/2 (b_l, Sec. 3.2)
* convergence_rows.txt - the ENO-MR rows of Tables 1DAdvectionConvergence5th,
  9th, 13th17th and 1DBurgersConvergence (Sec. 4.1, 4.2)

Values are copied verbatim as printed (typos included); the tests decide what
they mean.  Run once by hand:
``python tests/golden/extract_paper_tables.py <path of the paper's LaTeX source>``.
Nothing at test time reads the paper.
"""
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))

STENCIL_RE = re.compile(r"S_\{j(?:-(\d+))?\}\^\{j(?:\+(\d+))?\}")
FRAC_RE = re.compile(r"\\frac\{(-?\d+)\}\{(\d+)\}")


def table_blocks(lines, label):
    """Lines of the tabular environment that follows \\label{label}."""
    start = next(i for i, s in enumerate(lines) if "\\label{%s}" % label in s)
    end = next(i for i in range(start, len(lines)) if "\\end{tabular}" in lines[i])
    return start, lines[start:end]


def parse_coeff_table(lines, label):
    start, block = table_blocks(lines, label)
    out = []
    stencils = None
    for k, raw in enumerate(block):
        s = raw.strip()
        if s.startswith("$l$&"):
            stencils = []
            for cell in s.rstrip("\\").split("&")[1:]:
                mm = STENCIL_RE.search(cell)
                m = int(mm.group(1) or 0)
                n = int(mm.group(2) or 0)
                stencils.append((m, n))
            continue
        mrow = re.match(r"^(-?\d+)\s*&", s)
        if not mrow or stencils is None:
            continue
        l = int(mrow.group(1))
        cells = s.rstrip("\\").rstrip().rstrip("\\").split("&")[1:]
        for (m, n), cell in zip(stencils, cells):
            c = cell.strip().strip("$").strip()
            if not c:
                continue
            fm = FRAC_RE.search(c)
            if fm:
                num, den = int(fm.group(1)), int(fm.group(2))
            else:
                num, den = int(c), 1
            out.append((m, n, l, num, den, label.split(":")[1]))
    return out


def parse_convergence(lines, label, kind):
    start, block = table_blocks(lines, label)
    rows = []
    scheme = lam = alpha = None
    for k, raw in enumerate(block):
        s = raw.strip()
        hm = re.search(r"\\multicolumn\{4\}\{\|c\|\}\{([^$]+?),\$\\lambda=([^,$]+)(?:,\\alpha=(\d))?\$\}", s)
        if hm:
            # two multicolumn headers per line: left block and right block
            heads = re.findall(r"\\multicolumn\{4\}\{\|c\|\}\{([^$]+?),\$\\lambda=([^,$]+)(?:,\\alpha=(\d))?\$\}", s)
            scheme = heads
            continue
        dm = re.match(r"^(1/\d+)\s*&", s)
        if dm and scheme:
            cells = [c.strip() for c in s.rstrip("\\").split("&")]
            h = cells[0]
            vals = cells[1:]
            for side, (name, lam_s, alpha_s) in enumerate(scheme):
                if not name.startswith("ENO-MR"):
                    continue
                l1 = vals[4 * side + 0]
                linf = vals[4 * side + 2]
                lam_v = lam_s.replace("10^{", "1e").replace("}", "").replace("10^", "1e")
                rows.append((kind, name, lam_v, alpha_s or "-", h, l1, linf, label.split(":")[1]))
    return rows


def main():
    if len(sys.argv) != 2:
        sys.exit("usage: extract_paper_tables.py <path of the paper's LaTeX source>")
    paper = sys.argv[1]
    if not os.path.exists(paper):
        sys.exit("paper source not found at %s" % paper)
    with open(paper) as fh:
        lines = fh.read().splitlines()

    a_rows = parse_coeff_table(lines, "Table:Flux_reconstruction1") + \
        parse_coeff_table(lines, "Table:Flux_reconstruction2")
    b_rows = parse_coeff_table(lines, "Table:ISCoe1") + parse_coeff_table(lines, "Table:ISCoe2")

    hdr = ("# {what} as printed in H. Shen, arXiv 2311.15504, Sec. 3, {tables}.\n"
           "# Stencil S_(j-m)^(j+n) is written m n; columns: m n l numerator denominator table\n"
           "# Copied verbatim by extract_paper_tables.py (typos included).\n")
    with open(os.path.join(HERE, "a_coefficients.txt"), "w") as fh:
        fh.write(hdr.format(what="a_l of Eq. (ReconstructedFlux)",
                            tables="Tables Flux_reconstruction1 and Flux_reconstruction2"))
        for r in a_rows:
            fh.write("%d %d %d %d %d %s\n" % r)
    with open(os.path.join(HERE, "b_coefficients.txt"), "w") as fh:
        fh.write(hdr.format(what="b_l of Eq. (ISCoe)", tables="Tables ISCoe1 and ISCoe2"))
        for r in b_rows:
            fh.write("%d %d %d %d %d %s\n" % r)

    conv = []
    conv += parse_convergence(lines, "Table:1DAdvectionConvergence5th", "advection")
    conv += parse_convergence(lines, "Table:1DAdvectionConvergence9th", "advection")
    conv += parse_convergence(lines, "Table:1DAdvectionConvergence13th17th", "advection")
    conv += parse_convergence(lines, "Table:1DBurgersConvergence", "burgers")
    with open(os.path.join(HERE, "convergence_rows.txt"), "w") as fh:
        fh.write("# ENO-MR error rows printed in H. Shen, arXiv 2311.15504, Sec. 4.1 Tables\n"
                 "# 1DAdvectionConvergence5th/9th/13th17th (advection of lambda*sin^alpha(pi x),\n"
                 "# t=2) and Sec. 4.2 Table 1DBurgersConvergence (Burgers, t=0.1/lambda).\n"
                 "# The paper computed them in quadruple precision.\n"
                 "# columns: problem scheme lambda alpha h L1 Linf table\n")
        for r in conv:
            fh.write("%s %s %s %s %s %s %s %s\n" % r)
    print("a:", len(a_rows), "b:", len(b_rows), "convergence rows:", len(conv))


if __name__ == "__main__":
    main()
