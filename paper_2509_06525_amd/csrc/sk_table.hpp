// Slater-Koster two-centre table (Slater & Koster, Phys. Rev. 94, 1498 (1954),
// Table I) for s, p and d orbitals, in the arithmetic type T of the caller:
// the builders form blocks in double, the recurrence on displacement-only
// blocks forms them in the vector type.  Orbitals s, px, py, pz, dxy, dyz, dzx,
// dx2-y2, d3z2-r2; integrals v = {ss_sigma, sp_sigma, pp_sigma, pp_pi,
// sd_sigma, pd_sigma, pd_pi, dd_sigma, dd_pi, dd_delta}.
#pragma once

namespace tbk {

// The s-d row and the p-d block of the table for integrals v.
template <class T>
__device__ __forceinline__ void sk_sd_pd(const T *v, T l, T m, T n, T (&sdr)[5], T (&pd)[3][5]) {
    const T s3 = T(1.7320508075688772);
    const T l2 = l * l, m2 = m * m, n2 = n * n;
    const T sd = v[4], pds = v[5], pdp = v[6];
    const T q = n2 - T(0.5) * (l2 + m2), dlm = l2 - m2;
    sdr[0] = s3 * l * m * sd;
    sdr[1] = s3 * m * n * sd;
    sdr[2] = s3 * n * l * sd;
    sdr[3] = T(0.5) * s3 * dlm * sd;
    sdr[4] = q * sd;
    pd[0][0] = s3 * l2 * m * pds + m * (T(1.0) - T(2.0) * l2) * pdp;
    pd[0][1] = s3 * l * m * n * pds - T(2.0) * l * m * n * pdp;
    pd[0][2] = s3 * l2 * n * pds + n * (T(1.0) - T(2.0) * l2) * pdp;
    pd[0][3] = T(0.5) * s3 * l * dlm * pds + l * (T(1.0) - dlm) * pdp;
    pd[0][4] = l * q * pds - s3 * l * n2 * pdp;
    pd[1][0] = s3 * m2 * l * pds + l * (T(1.0) - T(2.0) * m2) * pdp;
    pd[1][1] = s3 * m2 * n * pds + n * (T(1.0) - T(2.0) * m2) * pdp;
    pd[1][2] = s3 * l * m * n * pds - T(2.0) * l * m * n * pdp;
    pd[1][3] = T(0.5) * s3 * m * dlm * pds - m * (T(1.0) + dlm) * pdp;
    pd[1][4] = m * q * pds - s3 * m * n2 * pdp;
    pd[2][0] = s3 * l * m * n * pds - T(2.0) * l * m * n * pdp;
    pd[2][1] = s3 * n2 * m * pds + m * (T(1.0) - T(2.0) * n2) * pdp;
    pd[2][2] = s3 * n2 * l * pds + l * (T(1.0) - T(2.0) * n2) * pdp;
    pd[2][3] = T(0.5) * s3 * n * dlm * pds - n * dlm * pdp;
    pd[2][4] = n * q * pds + s3 * n * (l2 + m2) * pdp;
}

// The Slater-Koster table: E[a][b] = <a_i|H|b_j> / f for direction cosines
// (l, m, n) from i to j.  The blocks with the lower angular momentum on the row
// side (and the equal-l blocks) come from the integrals vu of the ordered
// species pair (row, column), the others from the reversed pair's vl by
// E[b][a] = (-1)^(l_a + l_b) E'[a][b] (E' formed with vl; vl = vu for one
// species).  Only the first NORB rows and columns are formed.  SAME: vl is
// vu (one species), so the s-d and p-d pieces are formed once.
template <class T, int NORB, bool SAME = false>
__device__ __forceinline__ void sk_table(const T *vu, const T *vl, T l, T m, T n, T (&E)[NORB][NORB]) {
    const T *v = vu;
    const T s3 = T(1.7320508075688772);
    const T l2 = l * l, m2 = m * m, n2 = n * n;
    const T c[3] = {l, m, n};
    E[0][0] = v[0];
    for (int a = 0; a < 3; ++a) {
        E[0][1 + a] = c[a] * v[1];
        E[1 + a][0] = -c[a] * vl[1];
        for (int b = 0; b < 3; ++b) E[1 + a][1 + b] = c[a] * c[b] * v[2] + ((a == b ? T(1.0) : T(0.0)) - c[a] * c[b]) * v[3];
    }
    if constexpr (NORB == 9) {
        const T dds = v[7], ddp = v[8], ddd = v[9];
        const T q = n2 - T(0.5) * (l2 + m2), dlm = l2 - m2;
        T sdr[5], pd[3][5], sdl[5], pdl[3][5];
        sk_sd_pd<T>(vu, l, m, n, sdr, pd);
        if constexpr (SAME) {
            for (int a = 0; a < 5; ++a) {
                sdl[a] = sdr[a];
                for (int b = 0; b < 3; ++b) pdl[b][a] = pd[b][a];
            }
        } else {
            sk_sd_pd<T>(vl, l, m, n, sdl, pdl);
        }
        T dd[5][5];
        dd[0][0] = T(3.0) * l2 * m2 * dds + (l2 + m2 - T(4.0) * l2 * m2) * ddp + (n2 + l2 * m2) * ddd;
        dd[1][1] = T(3.0) * m2 * n2 * dds + (m2 + n2 - T(4.0) * m2 * n2) * ddp + (l2 + m2 * n2) * ddd;
        dd[2][2] = T(3.0) * n2 * l2 * dds + (n2 + l2 - T(4.0) * n2 * l2) * ddp + (m2 + n2 * l2) * ddd;
        dd[0][1] = T(3.0) * l * m2 * n * dds + l * n * (T(1.0) - T(4.0) * m2) * ddp + l * n * (m2 - T(1.0)) * ddd;
        dd[0][2] = T(3.0) * l2 * m * n * dds + m * n * (T(1.0) - T(4.0) * l2) * ddp + m * n * (l2 - T(1.0)) * ddd;
        dd[1][2] = T(3.0) * l * m * n2 * dds + l * m * (T(1.0) - T(4.0) * n2) * ddp + l * m * (n2 - T(1.0)) * ddd;
        dd[0][3] = T(1.5) * l * m * dlm * dds - T(2.0) * l * m * dlm * ddp + T(0.5) * l * m * dlm * ddd;
        dd[1][3] = T(1.5) * m * n * dlm * dds - m * n * (T(1.0) + T(2.0) * dlm) * ddp + m * n * (T(1.0) + T(0.5) * dlm) * ddd;
        dd[2][3] = T(1.5) * n * l * dlm * dds + n * l * (T(1.0) - T(2.0) * dlm) * ddp - n * l * (T(1.0) - T(0.5) * dlm) * ddd;
        dd[0][4] = s3 * (l * m * q * dds - T(2.0) * l * m * n2 * ddp + T(0.5) * l * m * (T(1.0) + n2) * ddd);
        dd[1][4] = s3 * (m * n * q * dds + m * n * (l2 + m2 - n2) * ddp - T(0.5) * m * n * (l2 + m2) * ddd);
        dd[2][4] = s3 * (l * n * q * dds + l * n * (l2 + m2 - n2) * ddp - T(0.5) * l * n * (l2 + m2) * ddd);
        dd[3][3] = T(0.75) * dlm * dlm * dds + (l2 + m2 - dlm * dlm) * ddp + (n2 + T(0.25) * dlm * dlm) * ddd;
        dd[3][4] = s3 * (T(0.5) * dlm * q * dds - n2 * dlm * ddp + T(0.25) * (T(1.0) + n2) * dlm * ddd);
        dd[4][4] = q * q * dds + T(3.0) * n2 * (l2 + m2) * ddp + T(0.75) * (l2 + m2) * (l2 + m2) * ddd;
        for (int a = 0; a < 5; ++a) {
            E[0][4 + a] = sdr[a];
            E[4 + a][0] = sdl[a];                      // d-s: even
            for (int b = 0; b < 3; ++b) {
                E[1 + b][4 + a] = pd[b][a];
                E[4 + a][1 + b] = -pdl[b][a];          // d-p: odd
            }
            for (int b = a; b < 5; ++b) {
                E[4 + a][4 + b] = dd[a][b];
                E[4 + b][4 + a] = dd[a][b];
            }
        }
    }
}

}  // namespace tbk
