# A CPU program in plain Python: the 19-point variable-coefficient Jacobi
# relaxation, written with its own names and its own arrangement of the
# terms. The front end must find its loops, screen them, derive the transfer
# sets and bind it to the library's nests by what it computes.


def relax(u, nxt, e, n_, t, diag, xy, yz, xz, w_, s_, b_, mask, src, steps, w):
    nk, nj, ni = u.shape
    for step in range(steps):
        err = 0.0
        for z in range(1, nk - 1):
            for y in range(1, nj - 1):
                for x in range(1, ni - 1):
                    acc = (src[z, y, x]
                           + e[z, y, x] * u[z, y, x + 1] + w_[z, y, x] * u[z, y, x - 1]
                           + n_[z, y, x] * u[z, y + 1, x] + s_[z, y, x] * u[z, y - 1, x]
                           + t[z, y, x] * u[z + 1, y, x] + b_[z, y, x] * u[z - 1, y, x]
                           + xy[z, y, x] * (u[z, y + 1, x + 1] - u[z, y + 1, x - 1])
                           - xy[z, y, x] * (u[z, y - 1, x + 1] - u[z, y - 1, x - 1])
                           + yz[z, y, x] * (u[z + 1, y + 1, x] + u[z - 1, y - 1, x]
                                            - u[z + 1, y - 1, x] - u[z - 1, y + 1, x])
                           + xz[z, y, x] * (u[z + 1, y, x + 1] - u[z - 1, y, x + 1]
                                            - u[z + 1, y, x - 1] + u[z - 1, y, x - 1]))
                    upd = mask[z, y, x] * (diag[z, y, x] * acc - u[z, y, x])
                    nxt[z, y, x] = u[z, y, x] + w * upd
        for z in range(1, nk - 1):
            for y in range(1, nj - 1):
                for x in range(1, ni - 1):
                    err += (nxt[z, y, x] - u[z, y, x]) ** 2 / (w * w)
        for z in range(1, nk - 1):
            for y in range(1, nj - 1):
                for x in range(1, ni - 1):
                    u[z, y, x] = nxt[z, y, x]
    return err, u
