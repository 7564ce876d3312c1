/*
 * drops_oracle.c -- plain CPU oracle of the drop diagnostics used in the
 * paper's results (sec. 4): drops as connected regions of the phase field,
 * their volumes V, the effective diameter D with (4 pi / 3)(D/2)^3 = V (the
 * drop-size PDF is a histogram of D/H), and the mass loss
 * l_loss = (m_t - m_0) / m_0 (the last is a ratio of two sums of C and has
 * no code here).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it; it shares no code with the GPU
 * library.
 *
 * Readings where the paper is silent (listed in the design notes):
 *   - a drop is a set of cells with C >= threshold (1/2: the mid-value of
 *     the two phases) connected through cell faces; periodic axes wrap,
 *     walls do not connect;
 *   - V = h^3 x (number of cells of the drop).
 *
 * The labelling is a breadth-first flood fill started from every unvisited
 * cell in increasing linear order (x fastest), so each drop's label is the
 * smallest linear index among its cells; cells below the threshold get -1.
 */
#include <stdint.h>
#include <stdlib.h>

/* bc[d]: 0 periodic, 1 wall.  Returns the number of drops, -1 on failure. */
int64_t oracle_label_drops(const int64_t n[3], const int bc[3], const double* C, double thr,
                           int64_t* label)
{
    const int64_t nx = n[0], ny = n[1], nz = n[2];
    const int64_t N = nx * ny * nz;
    int64_t* queue = malloc(sizeof(int64_t) * (N > 0 ? N : 1));
    if (!queue) return -1;
    for (int64_t p = 0; p < N; ++p) label[p] = -2;   /* unvisited */
    int64_t ndrops = 0;
    for (int64_t seed = 0; seed < N; ++seed) {
        if (label[seed] != -2) continue;
        if (!(C[seed] >= thr)) {
            label[seed] = -1;
            continue;
        }
        ++ndrops;
        int64_t head = 0, tail = 0;
        queue[tail++] = seed;
        label[seed] = seed;
        while (head < tail) {
            const int64_t p = queue[head++];
            const int64_t x = p % nx, y = (p / nx) % ny, z = p / (nx * ny);
            const int64_t c[3] = {x, y, z}, len[3] = {nx, ny, nz};
            const int64_t stride[3] = {1, nx, nx * ny};
            for (int d = 0; d < 3; ++d)
                for (int s = -1; s <= 1; s += 2) {
                    int64_t q = c[d] + s;
                    if (q < 0 || q >= len[d]) {
                        if (bc[d] != 0) continue;
                        q = (q + len[d]) % len[d];
                    }
                    const int64_t nb = p + (q - c[d]) * stride[d];
                    if (label[nb] != -2) continue;
                    if (C[nb] >= thr) {
                        label[nb] = seed;
                        queue[tail++] = nb;
                    } else {
                        label[nb] = -1;
                    }
                }
        }
    }
    free(queue);
    return ndrops;
}
