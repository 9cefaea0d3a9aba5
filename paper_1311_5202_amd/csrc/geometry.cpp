// Nystrom discretisation on curved quadratic triangles (paper section 2.2):
// the nodes of each element are the six points of a degree-4 symmetric Gauss
// rule on the triangle, so N = 6 N_e.  Rule: D. A. Dunavant, "High degree
// efficient symmetrical Gaussian quadrature rules for the triangle" (1985),
// degree 4, two three-point orbits.
//
// Node numbering inside an element (an interface convention shared with the
// callers): g = 0,1,2 at reference coordinates (a,a), (1-2a,a), (a,1-2a);
// g = 3,4,5 at (b,b), (1-2b,b), (b,1-2b).  Element geometric nodes: corners
// 0,1,2 at (0,0), (1,0), (0,1), mid-edge nodes 3,4,5 on edges (0,1), (1,2),
// (2,0).  The normal used by the method points into the body:
// n = -(y_,1 x y_,2)/|y_,1 x y_,2| for corners ordered counter-clockwise
// when seen from the acoustic domain.
#include <cmath>

#include "plan.hpp"

namespace fdbem {

namespace {
constexpr double kA = 0.445948490915965;
constexpr double kB = 0.091576213509771;
constexpr double kWA = 0.223381589678011 * 0.5;  // reference triangle area 1/2
constexpr double kWB = 0.109951743655322 * 0.5;
}  // namespace

void gauss6(double xi[6][2], double wq[6])
{
    const double a = kA, b = kB;
    const double pts[6][2] = {{a, a}, {1 - 2 * a, a}, {a, 1 - 2 * a}, {b, b}, {1 - 2 * b, b}, {b, 1 - 2 * b}};
    for (int g = 0; g < 6; ++g) {
        xi[g][0] = pts[g][0];
        xi[g][1] = pts[g][1];
        wq[g] = g < 3 ? kWA : kWB;
    }
}

void p2_shape(double s, double t, double N[6], double dNs[6], double dNt[6])
{
    const double L0 = 1.0 - s - t, L1 = s, L2 = t;
    N[0] = L0 * (2 * L0 - 1);
    N[1] = L1 * (2 * L1 - 1);
    N[2] = L2 * (2 * L2 - 1);
    N[3] = 4 * L0 * L1;
    N[4] = 4 * L1 * L2;
    N[5] = 4 * L2 * L0;
    dNs[0] = -(4 * L0 - 1);
    dNs[1] = 4 * L1 - 1;
    dNs[2] = 0;
    dNs[3] = 4 * (L0 - L1);
    dNs[4] = 4 * L2;
    dNs[5] = -4 * L2;
    dNt[0] = -(4 * L0 - 1);
    dNt[1] = 0;
    dNt[2] = 4 * L2 - 1;
    dNt[3] = -4 * L1;
    dNt[4] = 4 * L1;
    dNt[5] = 4 * (L0 - L2);
}

void element_eval(const double *el, double s, double t, double y[3], double ys[3], double yt[3])
{
    double N[6], dNs[6], dNt[6];
    p2_shape(s, t, N, dNs, dNt);
    for (int d = 0; d < 3; ++d) {
        y[d] = ys[d] = yt[d] = 0;
        for (int a = 0; a < 6; ++a) {
            y[d] += N[a] * el[3 * a + d];
            ys[d] += dNs[a] * el[3 * a + d];
            yt[d] += dNt[a] * el[3 * a + d];
        }
    }
}

void nystrom_nodes(int64_t n_elem, const double *elem, double *pts, double *nrm, double *w)
{
    double xi[6][2], wq[6];
    gauss6(xi, wq);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n_elem; ++e) {
        const double *el = elem + 18 * e;
        for (int g = 0; g < 6; ++g) {
            double y[3], ys[3], yt[3];
            element_eval(el, xi[g][0], xi[g][1], y, ys, yt);
            const double c[3] = {ys[1] * yt[2] - ys[2] * yt[1], ys[2] * yt[0] - ys[0] * yt[2],
                                 ys[0] * yt[1] - ys[1] * yt[0]};
            const double J = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
            const int64_t j = 6 * e + g;
            for (int d = 0; d < 3; ++d) {
                pts[3 * j + d] = y[d];
                nrm[3 * j + d] = -c[d] / J;
            }
            w[j] = wq[g] * J;
        }
    }
}

}  // namespace fdbem
