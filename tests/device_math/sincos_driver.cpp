// Host build of the device sine/cosine helpers (device.hpp): the largest absolute error of
// sincos_angle over every FP32 heading step of [-pi, pi] on a 2^23-point grid and of
// sincos_turn over every Box-Muller uniform (2m + 1) 2^-24, against the C library's FP64
// sin and cos.  Prints "angle <err> turn <err>" in units of 2^-24.
#include <cmath>
#include <cstdio>

#include "device.hpp"

int main() {
    using cuesim::sincos_angle;
    using cuesim::sincos_turn;
    double e_angle = 0.0, e_turn = 0.0;
    const int half = 1 << 22;
    for (int k = -half; k <= half; ++k) {
        const float th = (float)(M_PI * k / (double)half);
        float s, c;
        sincos_angle(th, s, c);
        e_angle = std::fmax(e_angle, std::fabs(s - std::sin((double)th)));
        e_angle = std::fmax(e_angle, std::fabs(c - std::cos((double)th)));
    }
    for (int m = 0; m < (1 << 23); ++m) {
        const float u = (float)m * 0x1p-23f + 0x1p-24f;
        float s, c;
        sincos_turn(u, s, c);
        e_turn = std::fmax(e_turn, std::fabs(s - std::sin(2.0 * M_PI * (double)u)));
        e_turn = std::fmax(e_turn, std::fabs(c - std::cos(2.0 * M_PI * (double)u)));
    }
    std::printf("angle %.4f turn %.4f\n", e_angle / 0x1p-24, e_turn / 0x1p-24);
    return 0;
}
