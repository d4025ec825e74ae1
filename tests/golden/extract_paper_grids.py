"""Write the paper's printed 2-D CGL sparse grids to text fixtures.

Recipe only (run by hand where the paper's LaTeX source is available); the
fixtures it writes are committed next to it.  Fig. 3 of Kang & Wilcox (Sec.
3.2, the CGL sparse grids for q = 6 and q = 8) prints every grid point as a
pgfplots table.  The data are plotted on [-1, 1]^2 although the caption says
[0, 1]^2; the fixtures keep the printed numbers and the tests map them with
xi = (x + 1) / 2.

Usage: python tests/golden/extract_paper_grids.py <LaTeX source of the paper>
"""
import os
import re
import sys


def main(path):
    text = open(path).read()
    start = text.index(r"\label{CGL}")
    tables = re.findall(r"table\[row sep=crcr\]\{(.*?)\};", text[start:], flags=re.S)[:2]
    out_dir = os.path.dirname(os.path.abspath(__file__))
    for q, body in zip((6, 8), tables):
        rows = [r.strip() for r in body.split(r"\\") if r.strip()]
        pts = [tuple(float(v) for v in r.split()) for r in rows]
        fn = os.path.join(out_dir, "paper_cgl_2d_q%d.txt" % q)
        with open(fn, "w") as f:
            f.write("# Kang & Wilcox, Sec. 3.2, Fig. 3 (CGL sparse grid, d=2, q=%d), "
                    "printed on [-1,1]^2; %d points\n" % (q, len(pts)))
            for x, y in pts:
                f.write("%r %r\n" % (x, y))
        print(fn, len(pts))


if __name__ == "__main__":
    if len(sys.argv) != 2:
        sys.exit("usage: extract_paper_grids.py <LaTeX source of the paper>")
    main(sys.argv[1])
