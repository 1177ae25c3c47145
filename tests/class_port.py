"""Host port of the library's symbolic class choice (tier geometry, table
sizes, smallest tier that holds the table and gives each lane at most
`work_per_lane` products), used by tests to predict which class each row
gets.  Mirrors the device function with the default options: products per
lane 16, LDS limit 64 KiB, no forced class."""
TIER_GLOBAL = 9
EMPTY = 255


def tier_bytes(t):
    return 256 << t


def tier_threads(t):
    if t <= 2:
        return 8 << t
    return 64 if t <= 4 else 128 if t == 5 else 256 if t == 6 else 512 if t == 7 else 1024


def pow2ceil(x):
    p = 1
    while p < x:
        p <<= 1
    return p


def sym_hash_slots(est, bound=False):
    need = (est * 4 + 2) // 3 if bound else est * 2
    return pow2ceil(max(need, 16))


def align8(b):
    return (b + 7) & ~7


def pick_tier(nbytes, work, work_per_lane=16, lds_limit=65536):
    if nbytes > lds_limit:
        return TIER_GLOBAL
    t = 0
    while t < TIER_GLOBAL - 1 and tier_bytes(t) < nbytes:
        t += 1
    if tier_bytes(t) < nbytes:
        return TIER_GLOBAL
    while t < TIER_GLOBAL - 1 and tier_threads(t) * work_per_lane < work and tier_bytes(t + 1) <= lds_limit:
        t += 1
    return t


def sym_class(ub, cmin, cmax, est_blocks, bound=False, work_per_lane=16):
    if ub <= 0:
        return EMPTY
    words = (cmax >> 5) - (cmin >> 5) + 1
    est = max(min(est_blocks, words), 1)
    bd = words * 4
    bh = sym_hash_slots(est, bound) * 8
    b2 = align8(((words + 31) // 32) * 8) + est * (6 if words <= 65536 else 8)
    mode, nbytes = 0, bd
    if b2 < nbytes:
        mode, nbytes = 2, b2
    if bh < nbytes:
        mode, nbytes = 1, bh
    t = pick_tier(nbytes, ub, work_per_lane)
    if t == TIER_GLOBAL or bd <= tier_bytes(t):
        mode = 0
    return mode * 10 + t
