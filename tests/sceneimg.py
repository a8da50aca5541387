"""Parser of the serialised scene image (host copy), for structural tests of the scene build."""
import numpy as np

HEADER = np.dtype([
    ("magic", "<u4"), ("version", "<u4"), ("n_tri", "<i4"), ("n_mat", "<i4"), ("n_bins", "<i4"), ("n_cells", "<i4"),
    ("grid", "<i4", 3), ("max_depth", "<i4"), ("lo", "<f4", 3), ("hi", "<f4", 3), ("sun", "<f4", 3),
    ("env_nonzero", "<i4"), ("off_planes", "<u8"), ("off_cells", "<u8"), ("off_nodes", "<u8"), ("off_ctris", "<u8"),
    ("off_gtris", "<u8"), ("off_mtype", "<u8"), ("off_thick", "<u8"), ("off_n", "<u8"), ("off_k", "<u8"),
    ("off_rho", "<u8"), ("off_lambda", "<u8"), ("off_sunE", "<u8"), ("off_env", "<u8"), ("n_nodes", "<u8"),
    ("n_refs", "<u8"), ("lambda_min_nm", "<f4"), ("lambda_max_nm", "<f4"), ("max_leaf", "<i4"), ("bins_pad", "<i4")])

EMPTY = 0xFFFFFFFF


class SceneImage:
    def __init__(self, buf: np.ndarray):
        self.buf = buf
        h = np.frombuffer(buf[:HEADER.itemsize].tobytes(), dtype=HEADER)[0]
        self.h = h
        g = [int(x) for x in h["grid"]]
        self.grid = g
        pl = np.frombuffer(buf, dtype="<f4", count=sum(g) + 3, offset=int(h["off_planes"]))
        self.planes = [pl[:g[0] + 1], pl[g[0] + 1:g[0] + g[1] + 2], pl[g[0] + g[1] + 2:]]
        self.cells = np.frombuffer(buf, dtype="<i4", count=4 * int(h["n_cells"]), offset=int(h["off_cells"])).reshape(-1, 4)
        nn = int(h["n_nodes"])
        self.node_u = np.frombuffer(buf, dtype="<u4", count=16 * nn, offset=int(h["off_nodes"])).reshape(nn, 16)
        nr = int(h["n_refs"])
        ct = np.frombuffer(buf, dtype="<f4", count=12 * nr, offset=int(h["off_ctris"])).reshape(nr, 3, 4)
        self.ctri_v = ct[:, :, :3]
        self.ctri_id = ct[:, 0, 3].view("<u4")
        self.ctri_mat = ct[:, 1, 3].view("<u4")
        nt = int(h["n_tri"])
        gt = np.frombuffer(buf, dtype="<f4", count=12 * nt, offset=int(h["off_gtris"])).reshape(nt, 3, 4)
        self.gtri_v = gt[:, :, :3]
        B = int(h["n_bins"])
        self.lam = np.frombuffer(buf, dtype="<f4", count=B, offset=int(h["off_lambda"]))

    def child(self, node, c):
        """(box lo[3], box hi[3], idx, cnt, step[3]) of child c (0..3) of a (global) 4-wide node of
        64 bytes: origin (3 floats) | exponents (bytes) ; child words ; lo.x hi.x lo.y hi.y bytes ;
        lo.z hi.z bytes. A bound is origin + q 2^(e - 127) (inner: node index; leaf: count << 27 |
        first triangle; EMPTY: no child); step is the grid spacing per axis."""
        u = self.node_u[node]
        origin = u[0:3].copy().view("<f4").astype(np.float64)
        e = int(u[3])
        step = np.array([2.0 ** (((e >> (8 * a)) & 255) - 127) for a in range(3)])
        q = [(int(u[8 + j]) >> (8 * c)) & 255 for j in range(6)]
        lo = origin + np.array([q[0], q[2], q[4]], dtype=np.float64) * step
        hi = origin + np.array([q[1], q[3], q[5]], dtype=np.float64) * step
        word = int(u[4 + c])
        if word == EMPTY:
            return lo, hi, EMPTY, 0, step
        return lo, hi, word & ((1 << 27) - 1), word >> 27, step

    def cell_of_point(self, p):
        idx = []
        for a in range(3):
            pl = self.planes[a]
            i = int(np.searchsorted(pl, p[a], side="right")) - 1
            idx.append(min(max(i, 0), len(pl) - 2))
        return (idx[2] * self.grid[1] + idx[1]) * self.grid[0] + idx[0]
