/* A CPU program in plain C99: the 19-point variable-coefficient Jacobi
 * relaxation with its own names (variable-length array parameters, the
 * scratch array a local VLA). The C front end reads it, and the test suite
 * also compiles and runs it as the original program. */

float solve(int nz, int ny, int nx, float v[nz][ny][nx], const float east[nz][ny][nx],
            const float north[nz][ny][nx], const float top[nz][ny][nx], const float inv_diag[nz][ny][nx],
            const float cxy[nz][ny][nx], const float cyz[nz][ny][nx], const float cxz[nz][ny][nx],
            const float west[nz][ny][nx], const float south[nz][ny][nx], const float bottom[nz][ny][nx],
            const float keep[nz][ny][nx], const float rhs[nz][ny][nx], int sweeps, float relax)
{
    float tmp[nz][ny][nx];
    float res = 0.0f;
    for (int it = 0; it < sweeps; ++it) {
        res = 0.0f;
        for (int z = 1; z < nz - 1; ++z)
            for (int y = 1; y < ny - 1; ++y)
                for (int x = 1; x < nx - 1; ++x) {
                    float s = east[z][y][x] * v[z][y][x + 1] + west[z][y][x] * v[z][y][x - 1]
                            + north[z][y][x] * v[z][y + 1][x] + south[z][y][x] * v[z][y - 1][x]
                            + top[z][y][x] * v[z + 1][y][x] + bottom[z][y][x] * v[z - 1][y][x]
                            + cxy[z][y][x] * (v[z][y + 1][x + 1] - v[z][y - 1][x + 1]
                                              - v[z][y + 1][x - 1] + v[z][y - 1][x - 1])
                            + cyz[z][y][x] * (v[z + 1][y + 1][x] - v[z + 1][y - 1][x]
                                              - v[z - 1][y + 1][x] + v[z - 1][y - 1][x])
                            + cxz[z][y][x] * (v[z + 1][y][x + 1] - v[z + 1][y][x - 1]
                                              - v[z - 1][y][x + 1] + v[z - 1][y][x - 1])
                            + rhs[z][y][x];
                    float d = (inv_diag[z][y][x] * s - v[z][y][x]) * keep[z][y][x];
                    tmp[z][y][x] = v[z][y][x] + relax * d;
                }
        for (int z = 1; z < nz - 1; ++z)
            for (int y = 1; y < ny - 1; ++y)
                for (int x = 1; x < nx - 1; ++x) {
                    float r = (tmp[z][y][x] - v[z][y][x]) / relax;
                    res += r * r;
                }
        for (int z = 1; z < nz - 1; ++z)
            for (int y = 1; y < ny - 1; ++y)
                for (int x = 1; x < nx - 1; ++x)
                    v[z][y][x] = tmp[z][y][x];
    }
    return res;
}
