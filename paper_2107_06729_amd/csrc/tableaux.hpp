// Butcher tableaux of the explicit methods named in Sec. II (Eq. (3)-(4)),
// coefficients from the publications the paper cites (refs. [26]-[31]).
// b is the propagated weight vector (c_k of Eq. (3)), bh the embedded one
// (c^_k), a the stage matrix (b_{k lambda} of Eq. (4)), c the nodes (a_k).
// The propagated solution follows the paper's naming: RKF45 and RKCK45
// propagate order 4, RKDP54 and RKF56 order 5, RK23 order 3, Heun order 2.
#pragma once

namespace llgx {

struct Tableau {
    const char* name;
    int S;            // stages
    int order;        // n, propagated
    int order_hat;    // n^, embedded (0: none)
    bool fsal;        // last stage at c = 1 with a-row = b
    double c[8];
    double a[8][8];
    double b[8];
    double bh[8];
    bool multistep;   // ABM2: stepped by its own predictor-corrector path, not by a, b
};

// clang-format off
static const Tableau TAB_RK4 = {"RK4", 4, 4, 0, false,
    {0, 0.5, 0.5, 1},
    {{0}, {0.5}, {0, 0.5}, {0, 0, 1}},
    {1.0 / 6, 1.0 / 3, 1.0 / 3, 1.0 / 6}, {0}};

static const Tableau TAB_HEUN = {"HEUN", 2, 2, 1, false,
    {0, 1},
    {{0}, {1}},
    {0.5, 0.5}, {1, 0}};

static const Tableau TAB_RK23 = {"RK23", 4, 3, 2, true,
    {0, 0.5, 0.75, 1},
    {{0}, {0.5}, {0, 0.75}, {2.0 / 9, 1.0 / 3, 4.0 / 9}},
    {2.0 / 9, 1.0 / 3, 4.0 / 9, 0}, {7.0 / 24, 0.25, 1.0 / 3, 0.125}};

static const Tableau TAB_RKF45 = {"RKF45", 6, 4, 5, false,
    {0, 0.25, 3.0 / 8, 12.0 / 13, 1, 0.5},
    {{0},
     {0.25},
     {3.0 / 32, 9.0 / 32},
     {1932.0 / 2197, -7200.0 / 2197, 7296.0 / 2197},
     {439.0 / 216, -8, 3680.0 / 513, -845.0 / 4104},
     {-8.0 / 27, 2, -3544.0 / 2565, 1859.0 / 4104, -11.0 / 40}},
    {25.0 / 216, 0, 1408.0 / 2565, 2197.0 / 4104, -0.2, 0},
    {16.0 / 135, 0, 6656.0 / 12825, 28561.0 / 56430, -9.0 / 50, 2.0 / 55}};

static const Tableau TAB_RKCK45 = {"RKCK45", 6, 4, 5, false,
    {0, 0.2, 0.3, 0.6, 1, 7.0 / 8},
    {{0},
     {0.2},
     {3.0 / 40, 9.0 / 40},
     {0.3, -0.9, 1.2},
     {-11.0 / 54, 2.5, -70.0 / 27, 35.0 / 27},
     {1631.0 / 55296, 175.0 / 512, 575.0 / 13824, 44275.0 / 110592, 253.0 / 4096}},
    {2825.0 / 27648, 0, 18575.0 / 48384, 13525.0 / 55296, 277.0 / 14336, 0.25},
    {37.0 / 378, 0, 250.0 / 621, 125.0 / 594, 0, 512.0 / 1771}};

static const Tableau TAB_RKDP54 = {"RKDP54", 7, 5, 4, true,
    {0, 0.2, 0.3, 0.8, 8.0 / 9, 1, 1},
    {{0},
     {0.2},
     {3.0 / 40, 9.0 / 40},
     {44.0 / 45, -56.0 / 15, 32.0 / 9},
     {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729},
     {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656},
     {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0},
    {5179.0 / 57600, 0, 7571.0 / 16695, 393.0 / 640, -92097.0 / 339200, 187.0 / 2100, 1.0 / 40}};

static const Tableau TAB_RKF56 = {"RKF56", 8, 5, 6, false,
    {0, 1.0 / 6, 4.0 / 15, 2.0 / 3, 0.8, 1, 0, 1},
    {{0},
     {1.0 / 6},
     {4.0 / 75, 16.0 / 75},
     {5.0 / 6, -8.0 / 3, 2.5},
     {-1.6, 144.0 / 25, -4, 16.0 / 25},
     {361.0 / 320, -3.6, 407.0 / 128, -11.0 / 80, 55.0 / 128},
     {-11.0 / 640, 0, 11.0 / 256, -11.0 / 160, 11.0 / 256, 0},
     {93.0 / 640, -3.6, 803.0 / 256, -11.0 / 160, 99.0 / 256, 0, 1}},
    {31.0 / 384, 0, 1125.0 / 2816, 9.0 / 32, 125.0 / 768, 5.0 / 66, 0, 0},
    {7.0 / 1408, 0, 1125.0 / 2816, 9.0 / 32, 125.0 / 768, 0, 5.0 / 66, 5.0 / 66}};
// Adams-Bashforth-Moulton, 2nd order (ref. [32]): PECE with a variable-step
// AB2 predictor and the trapezoidal corrector, two evaluations per step; the
// entries below only carry its name and orders (propagated 2, Milne estimate
// of the corrector's error: exponent 1/3 in Eq. (5)).
static const Tableau TAB_ABM2 = {"ABM2", 2, 2, 2, false, {0, 1}, {{0}, {1}}, {0.5, 0.5}, {1, 0}, true};
// clang-format on

inline const Tableau* tableau_for(int method) {
    switch (method) {
        case 0: return &TAB_RK4;
        case 1: return &TAB_RKF45;
        case 2: return &TAB_RKCK45;
        case 3: return &TAB_RKDP54;
        case 4: return &TAB_HEUN;
        case 5: return &TAB_RK23;
        case 6: return &TAB_RKF56;
        case 7: return &TAB_ABM2;
        default: return nullptr;
    }
}

}  // namespace llgx
