"""The iteration counts printed in Tables 3 and 4 (Section 7.2) for the
CANT-mx-2-2-l and BRIDGE-mx-2-2-l problems, mx in {2, 4, 6, 8}, l in
{5, 6, 7}, and the non-default PBM parameters their footnotes name.

Each entry: m, n (free displacement DOFs), the IP columns (iterations,
MINRES; None where the table has no entry because IP failed), the PBM
columns (outer iterations, Newton steps, MINRES), the footnote flags and,
for the bridges at l = 7, the res_PBM value at which the stalled run was
accepted.

Footnote flags (Section 7.2, the paragraph after the tables):
  1: gamma = beta = 0.5 instead of 0.3 (for CANT-8-2-2-7 together with the
     initial eps_MR = 1e-5 sqrt(n), which Table 3's footnote lists under 1);
  2: initial eps_MR = 1e-5 sqrt(n);
  3: initial eps_MR = 1e-5 sqrt(n) and eps_NWT = 0.1.
"""

CANT = {
    "CANT-2-2-2-5": (32768, 104544, (31, 368), (16, 50, 175), ()),
    "CANT-4-2-2-5": (65536, 209088, (28, 570), (15, 57, 153), ()),
    "CANT-6-2-2-5": (98304, 313632, (26, 467), (14, 45, 84), ()),
    "CANT-8-2-2-5": (131072, 418176, (27, 489), (14, 45, 115), ()),
    "CANT-2-2-2-6": (262144, 811200, (46, 1195), (18, 60, 141), ()),
    "CANT-4-2-2-6": (524288, 1622400, (42, 2465), (17, 59, 118), ()),
    "CANT-6-2-2-6": (786432, 2433600, (39, 1015), (17, 66, 157), ()),
    "CANT-8-2-2-6": (1048576, 3244800, (39, 1079), (16, 57, 88), ()),
    "CANT-2-2-2-7": (2097152, 6390144, (71, 2383), (22, 66, 70), ()),
    "CANT-4-2-2-7": (4194304, 12780288, (54, 3543), (20, 57, 67), ()),
    "CANT-6-2-2-7": (6291456, 19170432, (57, 2667), (19, 60, 68), ()),
    "CANT-8-2-2-7": (8388608, 25560576, (58, 2335), (29, 64, 100), (1, 2)),
}

BRIDGE = {
    "BRIDGE-2-2-2-5": (32768, 107799, (24, 387), (15, 49, 220), ()),
    "BRIDGE-4-2-2-5": (65536, 212343, (25, 590), (14, 45, 155), ()),
    "BRIDGE-6-2-2-5": (98304, 316887, (26, 778), (15, 55, 309), ()),
    "BRIDGE-8-2-2-5": (131072, 421431, (25, 1050), (13, 47, 184), ()),
    "BRIDGE-2-2-2-6": (262144, 823863, (41, 2029), (15, 56, 263), ()),
    "BRIDGE-4-2-2-6": (524288, 1635063, (50, 2965), (15, 57, 317), ()),
    "BRIDGE-6-2-2-6": (786432, 2446263, None, (15, 61, 466), ()),
    "BRIDGE-8-2-2-6": (1048576, 3257463, None, (15, 62, 592), ()),
    "BRIDGE-2-2-2-7": (2097152, 6440055, (91, 4744), (26, 109, 1134), (1,), 1.14e-4),
    "BRIDGE-4-2-2-7": (4194304, 12830199, None, (26, 99, 718), (1,), 2.68e-4),
    "BRIDGE-6-2-2-7": (6291456, 19220343, None, (25, 98, 743), (1, 3), 2.22e-4),
    "BRIDGE-8-2-2-7": (8388608, 25610487, None, (25, 97, 707), (1, 2), 1.17e-3),
}

TABLES = {**CANT, **BRIDGE}


def entry(name):
    """dict view of one table row"""
    row = TABLES[name]
    return dict(m=row[0], n=row[1], ip=row[2], pbm=row[3], flags=row[4],
                res_pbm=row[5] if len(row) > 5 else None)


def paper_overrides(name, n):
    """The option values the footnotes give for this problem (empty for the
    paper's defaults): beta/gamma, eps_mr0 (absolute), eps_nwt0."""
    flags = entry(name)["flags"]
    o = {}
    if 1 in flags:
        o["beta"] = o["gamma"] = 0.5
    if 2 in flags or 3 in flags:
        o["eps_mr0"] = 1e-5 * n ** 0.5
    if 3 in flags:
        o["eps_nwt0"] = 0.1
    return o
